"""GPU Jacobi-PCG and mixed-precision refinement against the oracle."""
import math

import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def check_against_oracle(orc, ref, res, ores, b, rtol, lam_min):
    assert res.status == 0 and ores.status == 0
    assert res.relres <= rtol * (1 + 1e-3)
    assert abs(res.iters - ores.iters) <= max(2, math.ceil(0.01 * ores.iters))
    x = host(res.x)
    r_gpu = np.linalg.norm(b - orc.spmv(ref, x))
    r_ref = np.linalg.norm(b - orc.spmv(ref, ores.x))
    assert np.linalg.norm(x - ores.x) <= (r_gpu + r_ref) / lam_min * (1 + 1e-6)


def test_config1_cg(orc):
    spx = require_gpu()
    prob, _, b = W.config1()
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg(ref, b, 1e-8)
    res = A.cg_solve(dev(b), rtol=1e-8)
    print(f"config1 cg: gpu {res.iters} it relres {res.relres:.3e}; oracle {ores.iters} it", flush=True)
    # lambda_min: identity rows give 1, interior lowest mode from the closed form
    c = math.cos(math.pi / 63)
    lam_min = min(1.0, (8 - 4 * c - 4 * c * c) / 3)
    check_against_oracle(orc, ref, res, ores, b, 1e-8, lam_min)


@pytest.mark.parametrize("variant,blocks,vblocks,quad", [(1, 0, 0, 1), (2, 0, 0, 1), (2, 37, 5, 1),
                                                        (1, 2048, 3000, 1), (2, 0, 0, 0),
                                                        (3, 0, 0, 0), (3, 37, 5, 0), (4, 0, 0, 0),
                                                        (4, 37, 5, 1), (2, 777, 1500, 0)])
def test_config1_cg_shapes(orc, variant, blocks, vblocks, quad):
    spx = require_gpu()
    prob, _, b = W.config1()
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SPMV_VARIANT, variant)
    A.set_option(spx.OPT_SOLVER_BLOCKS, blocks)
    A.set_option(spx.OPT_VECTOR_BLOCKS, vblocks)
    A.set_option(spx.OPT_QUAD_LOADS, quad)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg(ref, b, 1e-8)
    res = A.cg_solve(dev(b), rtol=1e-8)
    c = math.cos(math.pi / 63)
    check_against_oracle(orc, ref, res, ores, b, 1e-8, min(1.0, (8 - 4 * c - 4 * c * c) / 3))
    m = A.cg_solve_mixed(dev(b), rtol_outer=1e-10, rtol_inner=1e-4)
    assert m.status == 0 and m.relres <= 1e-10


@pytest.mark.parametrize("rows", [32, 64, 128, 256])
def test_pipelined_walk_is_bitwise_identical(rows):
    spx = require_gpu()
    N = 14
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(4).standard_normal(N**3)))
    A = assemble(spx, prob)
    b = dev(np.random.default_rng(5).uniform(-1, 1, prob.n))
    A.set_option(spx.OPT_ROWS_PER_BLOCK, rows)
    A.set_option(spx.OPT_ROWS_PER_BLOCK_F32, rows)
    outs = []
    for pipe in (1, 0):
        A.set_option(spx.OPT_PIPELINE, pipe)
        r = A.cg_solve(b, rtol=1e-10)
        m = A.cg_solve_mixed(b, rtol_outer=1e-10, rtol_inner=1e-4)
        outs.append((r.iters, host(r.x), m.inner, host(m.x)))
    assert outs[0][0] == outs[1][0] and outs[0][2] == outs[1][2]
    assert np.array_equal(bits(outs[0][1]), bits(outs[1][1]))
    assert np.array_equal(bits(outs[0][3]), bits(outs[1][3]))


@pytest.mark.parametrize("rows", [32, 64])
def test_dma_walk_matches_stream_walk_bitwise(rows):
    """Same products, same row order, same partial order: the DMA staging
    changes how bytes reach LDS, not the arithmetic."""
    spx = require_gpu()
    N = 14
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(6).standard_normal(N**3)))
    A = assemble(spx, prob)
    b = dev(np.random.default_rng(7).uniform(-1, 1, prob.n))
    outs = []
    for variant in (2, 3):
        A.set_option(spx.OPT_SPMV_VARIANT, variant)
        A.set_option(spx.OPT_ROWS_PER_BLOCK, rows)
        A.set_option(spx.OPT_ROWS_PER_BLOCK_F32, rows)
        assert A.get_option(spx.OPT_SPMV_VARIANT) == variant
        r = A.cg_solve(b, rtol=1e-10)
        m = A.cg_solve_mixed(b, rtol_outer=1e-10, rtol_inner=1e-4)
        y = A.matmult(b)
        outs.append((r.iters, host(r.x), m.inner, host(m.x), host(y)))
    assert outs[0][0] == outs[1][0] and outs[0][2] == outs[1][2]
    for k in (1, 3, 4):
        assert np.array_equal(bits(outs[0][k]), bits(outs[1][k]))


def test_cg_check_every_does_not_change_the_result(orc):
    spx = require_gpu()
    prob, _, b = W.config1()
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SMALL_SOLVE, 0)  # the multi-workgroup path polls
    A.set_option(spx.OPT_CG_VARIANT, 0)
    outs = [A.cg_solve(dev(b), rtol=1e-8, check_every=k) for k in (1, 7, 20, 1000)]
    for o in outs[1:]:
        assert o.iters == outs[0].iters
        assert np.array_equal(bits(host(o.x)), bits(host(outs[0].x)))


@pytest.mark.parametrize("N,dim", [(3, 2), (8, 2), (2, 3), (4, 3)])
def test_cg_dense_lu(orc, N, dim):
    spx = require_gpu()
    rng = np.random.default_rng(40 + N)
    prob = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    D = np.zeros((prob.n, prob.n))
    D[np.repeat(np.arange(prob.n), np.diff(ref.rowptr)), ref.col] = ref.val
    b = rng.uniform(-1, 1, prob.n)
    xs = np.linalg.solve(D, b)
    res = A.cg_solve(dev(b), rtol=1e-14, maxit=10000)
    assert res.status == 0
    assert np.linalg.norm(host(res.x) - xs) <= 1e-10 * np.linalg.norm(xs)


def test_cg_eigenmode_converges_in_one_step():
    spx = require_gpu()
    N = 10
    prob = W.q1_poisson(N, 2)
    A = assemble(spx, prob)
    M = N + 1
    node = np.arange(prob.n)
    v = np.sin(2 * math.pi * (node % M) / N) * np.sin(3 * math.pi * (node // M) / N)
    cx, cy = math.cos(2 * math.pi / N), math.cos(3 * math.pi / N)
    lam = (8 - 2 * cx - 2 * cy - 4 * cx * cy) / 3
    res = A.cg_solve(dev(v), rtol=1e-12, maxit=50)
    assert res.status == 0 and res.iters == 1
    assert np.max(np.abs(host(res.x) - v / lam)) <= 1e-12 * np.max(np.abs(v / lam))


def test_cg_status_codes():
    spx = require_gpu()
    # zero diagonal
    A = spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)), dev(np.array([1, 0, 1], np.int32)))
    A.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    assert A.cg_solve(dev(np.ones(2)), rtol=1e-8, maxit=10).status == spx.ZERO_DIAGONAL
    # indefinite: breakdown
    B = spx.coo_preallocate(2, dev(np.array([0, 1], np.int32)), dev(np.array([0, 1], np.int32)))
    B.set_values_coo(dev(np.array([1.0, -1.0])))
    assert B.cg_solve(dev(np.array([0.0, 1.0])), rtol=1e-8, maxit=10).status == spx.BREAKDOWN
    # iteration limit
    prob = W.q1_poisson(20, 2)
    C = assemble(spx, prob)
    b = np.random.default_rng(0).uniform(-1, 1, prob.n)
    r = C.cg_solve(dev(b), rtol=1e-12, maxit=3)
    assert r.status == spx.NOT_CONVERGED and r.iters == 3 and r.relres < 1.0
    r = C.cg_solve(dev(b), rtol=1e-12, maxit=0)
    assert r.status == spx.NOT_CONVERGED and r.iters == 0
    # b = 0
    r = C.cg_solve(dev(np.zeros(prob.n)), rtol=1e-8)
    assert r.status == 0 and r.iters == 0 and np.all(host(r.x) == 0)
    # nonzero initial guess is honoured
    x0 = np.random.default_rng(1).uniform(-1, 1, prob.n)
    r = C.cg_solve(dev(b), x=dev(x0), rtol=1e-10)
    assert r.status == 0 and r.relres <= 1e-10 * 1.001


def test_transpose_solve_of_symmetric_matrix_is_identical():
    spx = require_gpu()
    N = 12
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(2).standard_normal(N**3)))
    A = assemble(spx, prob)
    b = dev(np.random.default_rng(3).uniform(-1, 1, prob.n))
    r1 = A.cg_solve(b, rtol=1e-10)
    r2 = A.cg_solve_transpose(b, rtol=1e-10)
    assert r1.iters == r2.iters
    assert np.array_equal(bits(host(r1.x)), bits(host(r2.x)))


@pytest.mark.parametrize("early", [False, True])
def test_mixed_precision_refinement(orc, early):
    spx = require_gpu()
    N = 16
    rng = np.random.default_rng(1)
    z = rng.standard_normal(N**3)
    prob = W.q1_poisson(N, 3, kappa=np.exp(z))
    b = rng.uniform(-1, 1, prob.n)
    A = assemble(spx, prob)
    assert A.get_option(spx.OPT_IR_EARLY_EXIT) == 0  # the literal inner rule by default
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    om = orc.pcg_mixed(ref, b, 1e-10, 1e-4, early_exit=early)
    o64 = orc.pcg(ref, b, 1e-12)
    res = A.cg_solve_mixed(dev(b), rtol_outer=1e-10, rtol_inner=1e-4, early_exit=early)
    assert A.get_option(spx.OPT_IR_EARLY_EXIT) == int(early)
    x = host(res.x)
    err = np.linalg.norm(x - o64.x) / np.linalg.norm(o64.x)
    print(f"mixed N={N} early_exit={early}: gpu outer {res.outer} inner {res.inner} relres "
          f"{res.relres:.3e}; oracle outer {om.outer} inner {om.inner}; error vs fp64 oracle "
          f"{err:.3e}", flush=True)
    assert res.status == 0 and res.relres <= 1e-10
    assert np.linalg.norm(b - orc.spmv(ref, x)) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    assert abs(res.outer - om.outer) <= 1
    assert abs(res.inner - om.inner) <= max(3, 0.05 * om.inner)
    assert err <= 1e-7


@pytest.mark.parametrize("variant", [0, 4])  # default walk, window walk
def test_graph_replay_is_bitwise_the_eager_solve(variant):
    """Each full poll chunk replayed as one HIP graph: same kernels, same
    arithmetic.  Several solves (each replays the graph many times) with eager
    work and synchronisation between them, every one against the eager
    result; then the transpose solve and the mixed solve's fp32 inner graph,
    and a change of vectors that forces a new capture."""
    spx = require_gpu()
    N = 14
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(8).standard_normal(N**3)))
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SMALL_SOLVE, 0)  # compare the graph with the same multi-workgroup kernels
    A.set_option(spx.OPT_CG_VARIANT, 0)  # the textbook form, the one graphs capture
    A.set_option(spx.OPT_SPMV_VARIANT, variant)
    b = dev(np.random.default_rng(9).uniform(-1, 1, prob.n))
    eager = A.cg_solve(b, rtol=1e-10, check_every=7)
    eager_t = A.cg_solve_transpose(b, rtol=1e-10, check_every=7)
    eager_m = A.cg_solve_mixed(b, rtol_outer=1e-10, rtol_inner=1e-4, check_every=7)
    A.set_option(spx.OPT_GRAPH, 1)
    assert A.get_option(spx.OPT_GRAPH) == 1
    for rep in range(4):
        y = host(A.matmult(b))  # eager work between replays
        g = A.cg_solve(b, rtol=1e-10, check_every=7)
        assert g.iters == eager.iters and g.status == eager.status
        assert np.array_equal(bits(host(g.x)), bits(host(eager.x))), rep
        assert np.all(np.isfinite(y))
    gt = A.cg_solve_transpose(b, rtol=1e-10, check_every=7)
    assert gt.iters == eager_t.iters and np.array_equal(bits(host(gt.x)), bits(host(eager_t.x)))
    for rep in range(2):
        gm = A.cg_solve_mixed(b, rtol_outer=1e-10, rtol_inner=1e-4, check_every=7)
        assert (gm.outer, gm.inner) == (eager_m.outer, eager_m.inner)
        assert np.array_equal(bits(host(gm.x)), bits(host(eager_m.x))), rep
    b2 = dev(np.random.default_rng(10).uniform(-1, 1, prob.n))
    A.set_option(spx.OPT_GRAPH, 0)
    e2 = A.cg_solve(b2, rtol=1e-10, check_every=5)
    A.set_option(spx.OPT_GRAPH, 1)
    g2 = A.cg_solve(b2, rtol=1e-10, check_every=5)
    assert g2.iters == e2.iters and np.array_equal(bits(host(g2.x)), bits(host(e2.x)))


@pytest.mark.parametrize("mode", [0, 2])
def test_one_workgroup_and_multi_workgroup_solves(orc, mode):
    """SPX_OPT_SMALL_SOLVE 2 (the whole CG in one workgroup) and 0 (three
    kernels per iteration) each against the oracle, dense LU, the eigenmode
    and the statuses."""
    spx = require_gpu()
    prob, _, b = W.config1()
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SMALL_SOLVE, mode)
    A.set_option(spx.OPT_CG_VARIANT, 0)
    assert A.get_option(spx.OPT_SMALL_SOLVE) == mode
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg(ref, b, 1e-8)
    res = A.cg_solve(dev(b), rtol=1e-8)
    c = math.cos(math.pi / 63)
    check_against_oracle(orc, ref, res, ores, b, 1e-8, min(1.0, (8 - 4 * c - 4 * c * c) / 3))
    rt = A.cg_solve_transpose(dev(b), rtol=1e-8)
    assert rt.iters == res.iters and np.array_equal(bits(host(rt.x)), bits(host(res.x)))
    for N, dim in ((8, 2), (4, 3)):
        rng = np.random.default_rng(50 + N)
        p = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
        M = assemble(spx, p)
        M.set_option(spx.OPT_SMALL_SOLVE, mode)
        M.set_option(spx.OPT_CG_VARIANT, 0)
        R = orc.assemble(p.n, p.i, p.j, p.v)
        D = np.zeros((p.n, p.n))
        D[np.repeat(np.arange(p.n), np.diff(R.rowptr)), R.col] = R.val
        bb = rng.uniform(-1, 1, p.n)
        xs = np.linalg.solve(D, bb)
        r = M.cg_solve(dev(bb), rtol=1e-14, maxit=10000)
        assert r.status == 0 and np.linalg.norm(host(r.x) - xs) <= 1e-10 * np.linalg.norm(xs)
    N = 10
    p = W.q1_poisson(N, 2)
    E = assemble(spx, p)
    E.set_option(spx.OPT_SMALL_SOLVE, mode)
    E.set_option(spx.OPT_CG_VARIANT, 0)
    Mg = N + 1
    node = np.arange(p.n)
    v = np.sin(2 * math.pi * (node % Mg) / N) * np.sin(3 * math.pi * (node // Mg) / N)
    r = E.cg_solve(dev(v), rtol=1e-12, maxit=50)
    assert r.status == 0 and r.iters == 1
    Z = spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)), dev(np.array([1, 0, 1], np.int32)))
    Z.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    Z.set_option(spx.OPT_SMALL_SOLVE, mode)
    Z.set_option(spx.OPT_CG_VARIANT, 0)
    assert Z.cg_solve(dev(np.ones(2)), rtol=1e-8, maxit=10).status == spx.ZERO_DIAGONAL
    B = spx.coo_preallocate(2, dev(np.array([0, 1], np.int32)), dev(np.array([0, 1], np.int32)))
    B.set_values_coo(dev(np.array([1.0, -1.0])))
    B.set_option(spx.OPT_SMALL_SOLVE, mode)
    B.set_option(spx.OPT_CG_VARIANT, 0)
    rb = B.cg_solve(dev(np.array([0.0, 1.0])), rtol=1e-8, maxit=10)
    assert rb.status == spx.BREAKDOWN and rb.iters == 0
    C = assemble(spx, W.q1_poisson(20, 2))
    C.set_option(spx.OPT_SMALL_SOLVE, mode)
    C.set_option(spx.OPT_CG_VARIANT, 0)
    bc = np.random.default_rng(0).uniform(-1, 1, C.n)
    r = C.cg_solve(dev(bc), rtol=1e-12, maxit=3)
    assert r.status == spx.NOT_CONVERGED and r.iters == 3 and r.relres < 1.0
    r = C.cg_solve(dev(bc), rtol=1e-12, maxit=0)
    assert r.status == spx.NOT_CONVERGED and r.iters == 0
    r = C.cg_solve(dev(np.zeros(C.n)), rtol=1e-8)
    assert r.status == 0 and r.iters == 0 and np.all(host(r.x) == 0)
    x0 = np.random.default_rng(1).uniform(-1, 1, C.n)
    r = C.cg_solve(dev(bc), x=dev(x0), rtol=1e-10)
    assert r.status == 0 and r.relres <= 1e-10 * 1.001
