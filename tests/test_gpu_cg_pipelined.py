"""GPU pipelined (Ghysels-Vanroose) Jacobi-PCG against the oracle's
pipelined CG, plus the properties it shares with the textbook form."""
import math

import numpy as np
import pytest

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def lam_min_config1():
    c = math.cos(math.pi / 63)
    return min(1.0, (8 - 4 * c - 4 * c * c) / 3)


def pl(spx, A):
    A.set_option(spx.OPT_CG_VARIANT, 2)
    assert A.get_option(spx.OPT_CG_VARIANT) == 2
    return A


def check_against_oracle(orc, ref, res, ores, b, rtol, lam_min):
    assert res.status == 0 and ores.status == 0
    assert res.relres <= rtol * (1 + 1e-3)
    assert abs(res.iters - ores.iters) <= max(2, math.ceil(0.01 * ores.iters))
    x = host(res.x)
    r_gpu = np.linalg.norm(b - orc.spmv(ref, x))
    r_ref = np.linalg.norm(b - orc.spmv(ref, ores.x))
    assert np.linalg.norm(x - ores.x) <= (r_gpu + r_ref) / lam_min * (1 + 1e-6)


@pytest.mark.parametrize("variant,blocks,vblocks", [(0, 0, 0), (1, 0, 0), (2, 37, 5),
                                                    (1, 2048, 3000), (3, 0, 0), (3, 37, 5),
                                                    (4, 0, 0), (4, 37, 5)])
def test_config1_pipelined(orc, variant, blocks, vblocks):
    spx = require_gpu()
    prob, _, b = W.config1()
    A = pl(spx, assemble(spx, prob))
    A.set_option(spx.OPT_SPMV_VARIANT, variant)
    A.set_option(spx.OPT_SOLVER_BLOCKS, blocks)
    A.set_option(spx.OPT_VECTOR_BLOCKS, vblocks)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg_pipelined(ref, b, 1e-8)
    res = A.cg_solve(dev(b), rtol=1e-8)
    print(f"config1 pipelined cg (variant {variant}): gpu {res.iters} it relres "
          f"{res.relres:.3e}; oracle {ores.iters} it", flush=True)
    check_against_oracle(orc, ref, res, ores, b, 1e-8, lam_min_config1())
    hs = orc.pcg(ref, b, 1e-8)
    assert abs(res.iters - hs.iters) <= max(2, math.ceil(0.01 * hs.iters))


@pytest.mark.parametrize("k", [1, 2, 5, 13])
def test_pipelined_fixed_steps_match_oracle(orc, k):
    """After a fixed k steps (no stopping test) the iterate equals the
    oracle's pipelined iterate to rounding."""
    spx = require_gpu()
    rng = np.random.default_rng(17)
    N = 12
    prob = W.q1_poisson(N, 3, kappa=np.exp(rng.standard_normal(N**3)))
    b = rng.uniform(-1, 1, prob.n)
    A = pl(spx, assemble(spx, prob))
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg_pipelined(ref, b, 1e-30, k)
    res = A.cg_solve(dev(b), rtol=1e-30, maxit=k)
    assert res.status == spx.NOT_CONVERGED and res.iters == k and ores.iters == k
    x = host(res.x)
    assert np.linalg.norm(x - ores.x) <= 1e-11 * k * np.linalg.norm(ores.x)


def test_pipelined_check_every_is_invisible():
    spx = require_gpu()
    prob, _, b = W.config1()
    A = pl(spx, assemble(spx, prob))
    outs = [A.cg_solve(dev(b), rtol=1e-8, check_every=k) for k in (1, 7, 20, 1000)]
    for o in outs[1:]:
        assert o.iters == outs[0].iters
        assert np.array_equal(bits(host(o.x)), bits(host(outs[0].x)))


@pytest.mark.parametrize("N,dim", [(3, 2), (8, 2), (2, 3), (4, 3)])
def test_pipelined_dense_lu(N, dim):
    spx = require_gpu()
    rng = np.random.default_rng(40 + N)
    prob = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
    A = pl(spx, assemble(spx, prob))
    rowptr, col, val = (host(t) for t in A.get_csr())
    D = np.zeros((prob.n, prob.n))
    D[np.repeat(np.arange(prob.n), np.diff(rowptr)), col] = val
    b = rng.uniform(-1, 1, prob.n)
    xs = np.linalg.solve(D, b)
    res = A.cg_solve(dev(b), rtol=1e-13, maxit=10000)
    assert res.status == 0
    assert np.linalg.norm(host(res.x) - xs) <= 1e-10 * np.linalg.norm(xs)


def test_pipelined_eigenmode_one_step():
    spx = require_gpu()
    N = 10
    prob = W.q1_poisson(N, 2)
    A = pl(spx, assemble(spx, prob))
    M = N + 1
    node = np.arange(prob.n)
    v = np.sin(2 * math.pi * (node % M) / N) * np.sin(3 * math.pi * (node // M) / N)
    cx, cy = math.cos(2 * math.pi / N), math.cos(3 * math.pi / N)
    lam = (8 - 2 * cx - 2 * cy - 4 * cx * cy) / 3
    res = A.cg_solve(dev(v), rtol=1e-12, maxit=50)
    assert res.status == 0 and res.iters == 1
    assert np.max(np.abs(host(res.x) - v / lam)) <= 1e-12 * np.max(np.abs(v / lam))


def test_pipelined_status_codes():
    spx = require_gpu()
    A = pl(spx, spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)),
                                     dev(np.array([1, 0, 1], np.int32))))
    A.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    assert A.cg_solve(dev(np.ones(2)), rtol=1e-8, maxit=10).status == spx.ZERO_DIAGONAL
    B = pl(spx, spx.coo_preallocate(2, dev(np.array([0, 1], np.int32)),
                                     dev(np.array([0, 1], np.int32))))
    B.set_values_coo(dev(np.array([1.0, -1.0])))
    r = B.cg_solve(dev(np.array([0.0, 1.0])), rtol=1e-8, maxit=10)
    assert r.status == spx.BREAKDOWN and r.iters == 0
    prob = W.q1_poisson(20, 2)
    C = pl(spx, assemble(spx, prob))
    b = np.random.default_rng(0).uniform(-1, 1, prob.n)
    r = C.cg_solve(dev(b), rtol=1e-12, maxit=3)
    assert r.status == spx.NOT_CONVERGED and r.iters == 3 and r.relres < 1.0
    r = C.cg_solve(dev(b), rtol=1e-12, maxit=0)
    assert r.status == spx.NOT_CONVERGED and r.iters == 0
    r = C.cg_solve(dev(np.zeros(prob.n)), rtol=1e-8)
    assert r.status == 0 and r.iters == 0 and np.all(host(r.x) == 0)
    x0 = np.random.default_rng(1).uniform(-1, 1, prob.n)
    r = C.cg_solve(dev(b), x=dev(x0), rtol=1e-10)
    assert r.status == 0 and r.relres <= 1e-10 * 1.001
    # the allocation-free entry point refuses this form
    with pytest.raises(spx.SpxError) as e:
        C.cg_solve_noalloc(dev(b), x=dev(np.zeros(prob.n)), rtol=1e-8)
    assert e.value.code == spx.INVALID_ARG


def test_pipelined_transpose_of_symmetric_is_identical():
    spx = require_gpu()
    N = 12
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(2).standard_normal(N**3)))
    A = pl(spx, assemble(spx, prob))
    b = dev(np.random.default_rng(3).uniform(-1, 1, prob.n))
    r1 = A.cg_solve(b, rtol=1e-10)
    r2 = A.cg_solve_transpose(b, rtol=1e-10)
    assert r1.iters == r2.iters
    assert np.array_equal(bits(host(r1.x)), bits(host(r2.x)))


def test_pipelined_profile_counts_two_kernels():
    spx = require_gpu()
    prob, _, b = W.config1()
    A = pl(spx, assemble(spx, prob))
    A.set_option(spx.OPT_PROFILE, 1)
    A.reset_profile()
    res = A.cg_solve(dev(b), rtol=1e-8)
    prof = A.get_profile()
    # iters + 1 products (the last one is overlapped with the reduction that
    # finds convergence) and iters updates
    assert prof["spmv_dot_f64"][1] == res.iters + 1
    assert prof["update_f64"][1] == res.iters
    assert prof["pupdate_f64"][1] == 0


def test_full_size_pipelined(orc):
    """128^3-node log-normal workload to 1e-10 against the oracle's pipelined
    CG (iteration window, true residual), and within 1% of the textbook
    form's iteration count."""
    spx = require_gpu()
    print("full-size pipelined: generating", flush=True)
    prob, b = W.config3(127)
    A = assemble(spx, prob)
    hs = A.cg_solve(dev(b), rtol=1e-10)
    A.set_option(spx.OPT_CG_VARIANT, 2)
    res = A.cg_solve(dev(b), rtol=1e-10)
    orc.set_threads(16)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg_pipelined(ref, b, 1e-10)
    xs = host(res.x)
    rel = np.linalg.norm(b - orc.spmv(ref, xs)) / np.linalg.norm(b)
    print(f"pipelined {res.iters} it relres {res.relres:.3e} (oracle spmv {rel:.3e}); oracle "
          f"pipelined {ores.iters} it; textbook {hs.iters} it", flush=True)
    assert hs.status == 0 and res.status == 0 and ores.status == 0
    assert res.relres <= 1e-10 * 1.001 and rel <= 1e-10 * 1.001
    assert abs(res.iters - ores.iters) <= max(2, math.ceil(0.01 * ores.iters))
    assert abs(res.iters - hs.iters) <= max(2, math.ceil(0.01 * hs.iters))
