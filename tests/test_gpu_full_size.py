"""The full-size 3-D workloads against the oracle, element by element.

128^3-node Q1 Poisson, 131,096,512 COO triplets, 55,742,968 entries:

* kappa = 1 (the SpMV/CG workload): the whole assembled CSR bitwise equal
  to the oracle's, MatMult and MatMultTranspose within 1e-12 componentwise
  (bitwise for the in-order walks), Jacobi-CG to 1e-10 within the iteration
  window and error bound of the oracle-matching rule.
* log-normal kappa (sigma = 1): FP64 CG to 1e-10 against the oracle under
  the same rule, and the FP32-inner / FP64-outer refinement (literal inner
  rule and early exit) against the oracle's refinement: true FP64 residual,
  outer and inner counts, and the error against the FP64 oracle solve at
  1e-12, printed for each result.

The oracle's symbolic stage runs once; both value sets reuse its maps.
"""
import math
import os
import time

import numpy as np
import pytest

from paper_2406_08646_amd import workloads as W
from gpu_util import bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu

N = 127


def say(msg):
    print(f"[full-size] {msg}", flush=True)


def q1_3d_interior_lambda_min(N):
    """Smallest eigenvalue of the kappa = 1 3-D Q1 operator on the interior
    nodes: the closed form h [8/3 - 2/3 (cx cy + cy cz + cx cz) - 2/3 cx cy cz]
    with c_d = cos(k_d pi / N), minimised over every mode k in [1, N-1]^3."""
    c = np.cos(np.arange(1, N) * math.pi / N)
    cx, cy, cz = c[:, None, None], c[None, :, None], c[None, None, :]
    lam = (8.0 / 3.0 - 2.0 / 3.0 * (cx * cy + cy * cz + cx * cz) - 2.0 / 3.0 * cx * cy * cz) / N
    return float(lam.min())


def iteration_window(it, ref):
    return abs(it - ref) <= max(2, math.ceil(0.01 * ref))


@pytest.fixture(scope="module")
def full(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))
    t = time.time()
    prob2, x, b2 = W.config2(N)
    prob3, b3 = W.config3(N)
    assert np.array_equal(prob2.i, prob3.i) and np.array_equal(prob2.j, prob3.j)
    say(f"workloads generated in {time.time() - t:.1f} s: n={prob2.n} ncoo={prob2.ncoo}")
    t = time.time()
    rowptr, col, jmap, perm = orc.coo_pattern(prob2.n, prob2.i, prob2.j)
    ref2 = orc.CsrMatrix(prob2.n, rowptr, col, orc.coo_values(jmap, perm, prob2.v), jmap, perm,
                         prob2.ncoo)
    ref3 = orc.CsrMatrix(prob2.n, rowptr, col, orc.coo_values(jmap, perm, prob3.v), jmap, perm,
                         prob2.ncoo)
    say(f"oracle assembly in {time.time() - t:.1f} s: nnz={ref2.nnz}")
    v3 = prob3.v
    del prob3
    return prob2, x, b2, v3, b3, ref2, ref3


def test_full_size_kappa1_assembly_products_cg(orc, full):
    spx = require_gpu()
    prob, x, b, _, _, ref, _ = full
    assert ref.nnz == (3 * (N + 1) - 2) ** 3
    A = spx.coo_preallocate(prob.n, dev(prob.i), dev(prob.j))
    A.set_values_coo(dev(prob.v))
    rowptr, col, val = (host(t) for t in A.get_csr())
    assert np.array_equal(rowptr, ref.rowptr) and np.array_equal(col, ref.col)
    assert np.array_equal(bits(val), bits(ref.val))
    jm, pm = (host(t) for t in A.get_coo_maps())
    assert np.array_equal(jm.astype(np.int64), ref.jmap) and np.array_equal(pm, ref.perm)
    say("assembly: rowptr, col, val, jmap, perm bitwise equal to the oracle")
    del rowptr, col, val, jm, pm

    y = host(A.matmult(dev(x)))
    yt = host(A.matmult_transpose(dev(x)))
    y_ref = orc.spmv(ref, x)
    yt_ref = orc.spmv_transpose(ref, x)
    scale = orc.abs_spmv(ref, x)
    assert np.all(np.abs(y - y_ref) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(yt - yt_ref) <= 1e-12 * orc.abs_spmv_transpose(ref, x) + 1e-300)
    walk = A.get_option(spx.OPT_SPMV_VARIANT)
    if walk in (2, 4):
        # the stream and window walks round each product and add a row's
        # products in entry order from +0.0, the oracle's arithmetic
        assert np.array_equal(bits(y), bits(y_ref))
    say(f"MatMult / MatMultTranspose within 1e-12 of the oracle (walk {walk}); max rel "
        f"{np.max(np.abs(y - y_ref) / (scale + 1e-300)):.2e}")

    t = time.time()
    ores = orc.pcg(ref, b, 1e-10)
    say(f"oracle CG: {ores.iters} iterations in {time.time() - t:.1f} s, relres {ores.relres:.3e}")
    res = A.cg_solve(dev(b), rtol=1e-10, check_every=20)
    xs = host(res.x)
    r_gpu = np.linalg.norm(b - orc.spmv(ref, xs))
    r_ref = np.linalg.norm(b - orc.spmv(ref, ores.x))
    lam_min = min(1.0, q1_3d_interior_lambda_min(N))
    err = np.linalg.norm(xs - ores.x)
    bound = (r_gpu + r_ref) / lam_min
    say(f"GPU CG: {res.iters} iterations, relres {res.relres:.3e} (oracle spmv "
        f"{r_gpu / np.linalg.norm(b):.3e}); ||x - x_ref|| = {err:.3e}, bound {bound:.3e} "
        f"(lambda_min {lam_min:.6e})")
    assert res.status == 0 and ores.status == 0
    assert res.relres <= 1e-10 * (1 + 1e-3)
    assert r_gpu <= 1e-10 * np.linalg.norm(b) * (1 + 1e-3)
    assert iteration_window(res.iters, ores.iters), (res.iters, ores.iters)
    assert err <= bound * (1 + 1e-6)
    A.destroy()


def test_full_size_lognormal_fp64_and_mixed(orc, full):
    """The precision workload.  lambda_min of the log-normal operator is at
    least min(1, kappa_min lambda_min(kappa = 1)): every element matrix is
    kappa_e times a positive semi-definite one, and the identity rows of the
    Dirichlet nodes do not depend on kappa."""
    spx = require_gpu()
    prob, _, _, v3, b, _, ref = full
    z = np.random.default_rng(1).standard_normal(N**3)
    lam_min = min(1.0, float(np.exp(z.min())) * q1_3d_interior_lambda_min(N))
    bn = np.linalg.norm(b)
    A = spx.coo_preallocate(prob.n, dev(prob.i), dev(prob.j))
    A.set_values_coo(dev(v3))
    val = host(A.get_csr()[2])
    assert np.array_equal(bits(val), bits(ref.val))
    del val

    t = time.time()
    o64 = orc.pcg(ref, b, 1e-12)
    o10 = orc.pcg(ref, b, 1e-10)
    say(f"oracle FP64 CG: 1e-12 in {o64.iters} iterations, 1e-10 in {o10.iters} "
        f"({time.time() - t:.1f} s)")
    assert o64.status == 0 and o10.status == 0
    x64 = o64.x
    x64n = np.linalg.norm(x64)

    g = A.cg_solve(dev(b), rtol=1e-10)
    xg = host(g.x)
    rg = np.linalg.norm(b - orc.spmv(ref, xg))
    r10 = np.linalg.norm(b - orc.spmv(ref, o10.x))
    err_g = np.linalg.norm(xg - o10.x)
    say(f"GPU FP64 CG: {g.iters} iterations, true relres {rg / bn:.3e}; ||x - x_ref|| {err_g:.3e} "
        f"<= {(rg + r10) / lam_min:.3e}; error vs the FP64 oracle at 1e-12 "
        f"{np.linalg.norm(xg - x64) / x64n:.3e}")
    assert g.status == 0 and rg <= 1e-10 * bn * (1 + 1e-3)
    assert iteration_window(g.iters, o10.iters), (g.iters, o10.iters)
    assert err_g <= (rg + r10) / lam_min * (1 + 1e-6)

    for early in (False, True):
        t = time.time()
        om = orc.pcg_mixed(ref, b, 1e-10, 1e-4, early_exit=early)
        tm = time.time() - t
        m = A.cg_solve_mixed(dev(b), rtol_outer=1e-10, rtol_inner=1e-4, early_exit=early)
        xm = host(m.x)
        rm = np.linalg.norm(b - orc.spmv(ref, xm))
        rom = np.linalg.norm(b - orc.spmv(ref, om.x))
        err = np.linalg.norm(xm - x64) / x64n
        err_o = np.linalg.norm(om.x - x64) / x64n
        tag = "early exit" if early else "literal inner rtol 1e-4"
        say(f"mixed ({tag}): GPU {m.outer} outer / {m.inner} inner, true relres {rm / bn:.3e}; "
            f"oracle {om.outer} / {om.inner} ({tm:.1f} s), relres {rom / bn:.3e}; "
            f"||x_mixed - x_oracle64|| / ||x_oracle64|| = {err:.3e} (oracle's own refinement "
            f"{err_o:.3e})")
        assert m.status == 0 and om.status == 0
        assert rm <= 1e-10 * bn * (1 + 1e-6)
        assert abs(m.outer - om.outer) <= 1
        assert abs(m.inner - om.inner) <= max(3, math.ceil(0.05 * om.inner))
        assert np.linalg.norm(xm - x64) <= (rm + np.linalg.norm(b - orc.spmv(ref, x64))) / lam_min
    A.destroy()
