"""spx_cg_solve_noalloc (the CG solve in the library's static scratch)
against spx_cg_solve on the same handle and inputs: the same kernels and
launch shapes, so the same iteration count and bitwise the same x; both
within the oracle-matching rule of the oracle's CG.  Calls in a row of
decreasing size share the scratch; the largest is the full 128^3-node
workload (n = SPX_NOALLOC_MAX_ROWS exactly), the smallest takes the
one-workgroup solve.  Sizes above the limit are refused before any launch."""
import ctypes
import math

import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def lam_min_q1(N, dim):
    """Smallest eigenvalue of the kappa = 1 Q1 operator: min(1, interior
    closed form minimised over every mode)."""
    c = np.cos(np.arange(1, N) * math.pi / N)
    if dim == 2:
        cx, cy = c[:, None], c[None, :]
        lam = (8 - 2 * cx - 2 * cy - 4 * cx * cy) / 3
    else:
        cx, cy, cz = c[:, None, None], c[None, :, None], c[None, None, :]
        lam = (8 / 3 - 2 / 3 * (cx * cy + cy * cz + cx * cz) - 2 / 3 * cx * cy * cz) / N
    return min(1.0, float(lam.min()))


def raw_noalloc(spx, A, b, x, rtol):
    """The entry point called through the C ABI with raw pointers."""
    lib = spx.load_library()
    it, rr = ctypes.c_int64(), ctypes.c_double()
    rc = lib.spx_cg_solve_noalloc(A.handle, ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), rtol, 100000, 20,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.byref(it), ctypes.byref(rr))
    return rc, it.value, rr.value


@pytest.mark.parametrize("form", [-1, 0, 1])
def test_noalloc_matches_cg_solve(orc, form):
    spx = require_gpu()
    cases = [(127, 3, 1e-10), (40, 3, 1e-10), (63, 2, 1e-8), (12, 2, 1e-8)]
    for N, dim, rtol in cases:
        if dim == 3 and N == 127:
            prob, _, b = W.config2(N)
        else:
            prob = W.q1_poisson(N, dim)
            b = np.random.default_rng(N).uniform(-1, 1, prob.n)
        print(f"noalloc: form {form} N={N} dim={dim} n={prob.n}", flush=True)
        A = assemble(spx, prob)
        A.set_option(spx.OPT_CG_VARIANT, form)
        bd = dev(b)
        ref = A.cg_solve(bd, rtol=rtol)
        x = torch.zeros_like(bd)
        rc, iters, relres = raw_noalloc(spx, A, bd, x, rtol)
        assert rc == 0, spx.load_library().spx_last_error()
        assert iters == ref.iters and relres == ref.relres
        assert np.array_equal(bits(host(x)), bits(host(ref.x)))
        # the same again through the binding, from a nonzero start
        x0 = dev(np.random.default_rng(1).uniform(-1, 1, prob.n))
        r0 = A.cg_solve(bd, x=x0.clone(), rtol=rtol)
        r1 = A.cg_solve_noalloc(bd, x=x0.clone(), rtol=rtol)
        assert r1.status == 0 and r1.iters == r0.iters
        assert np.array_equal(bits(host(r1.x)), bits(host(r0.x)))
        if prob.n <= 300000:
            oref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
            ores = orc.pcg(oref, b, rtol)
            xs = host(x)
            r_gpu = np.linalg.norm(b - orc.spmv(oref, xs))
            r_ref = np.linalg.norm(b - orc.spmv(oref, ores.x))
            assert abs(iters - ores.iters) <= max(2, math.ceil(0.01 * ores.iters))
            assert r_gpu <= rtol * np.linalg.norm(b) * (1 + 1e-3)
            assert np.linalg.norm(xs - ores.x) <= (r_gpu + r_ref) / lam_min_q1(N, dim) * (1 + 1e-6)
        A.destroy()


def test_noalloc_limits_and_statuses():
    spx = require_gpu()
    lib = spx.load_library()
    # one row above the limit: refused with a message, nothing launched
    n = spx.NOALLOC_MAX_ROWS + 1
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    A = spx.coo_preallocate(n, idx, idx)
    A.set_values_coo(torch.full((n,), 2.0, dtype=torch.float64, device="cuda"))
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    rc, _, _ = raw_noalloc(spx, A, b, x, 1e-10)
    assert rc == spx.INVALID_ARG
    assert b"exceed" in lib.spx_last_error()
    assert torch.all(x == 0)
    A.destroy()
    # a launch shape beyond the scratch's partials
    prob = W.q1_poisson(20, 2)
    B = assemble(spx, prob)
    B.set_option(spx.OPT_SOLVER_BLOCKS, 5000)
    bb = dev(np.ones(prob.n))
    rc, _, _ = raw_noalloc(spx, B, bb, torch.zeros_like(bb), 1e-8)
    assert rc == spx.INVALID_ARG
    B.set_option(spx.OPT_SOLVER_BLOCKS, 0)
    # the solver statuses come through unchanged
    r = B.cg_solve_noalloc(bb, x=torch.zeros_like(bb), rtol=1e-12, maxit=3)
    assert r.status == spx.NOT_CONVERGED and r.iters == 3
    Z = spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)), dev(np.array([1, 0, 1], np.int32)))
    Z.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    z = Z.cg_solve_noalloc(dev(np.ones(2)), x=dev(np.zeros(2)), rtol=1e-8, maxit=10)
    assert z.status == spx.ZERO_DIAGONAL
    with pytest.raises(ValueError):
        B.cg_solve_noalloc(bb, None)
