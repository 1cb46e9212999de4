"""Batched Jacobi-CG (one launch per phase for all systems, or one persistent
launch with a workgroup per system) and multi-RHS SpMM against the
oracle."""
import math

import numpy as np
import pytest
import torch

from paper_2406_08646_amd import autotune, workloads as W
from gpu_util import assemble, dev, host, require_gpu, spmv_within

pytestmark = pytest.mark.gpu


def check_systems(orc, probs, bs, x, iters, relres, rtol):
    off = 0
    for s, (p, b) in enumerate(zip(probs, bs)):
        xs = x[off:off + p.n]
        off += p.n
        A = orc.assemble(p.n, p.i, p.j, p.v)
        ref = orc.pcg(A, b, rtol)
        assert ref.status == 0
        assert relres[s] <= rtol * (1 + 1e-3), (s, relres[s])
        r = np.linalg.norm(b - orc.spmv(A, xs)) / np.linalg.norm(b)
        assert r <= rtol * (1 + 1e-3), (s, r)
        assert abs(iters[s] - ref.iters) <= max(2, math.ceil(0.01 * ref.iters)), (s, iters[s], ref.iters)
        # error bound with lambda_min of the 5-point operator bounded below by the smallest
        # coefficient times the constant-coefficient closed form
        L = p.grid
        cmin = np.min(np.abs(p.v))  # every edge/face coefficient appears as +-c
        lam_min = cmin * (4 - 4 * math.cos(math.pi / (L + 1)))
        rr = np.linalg.norm(b - orc.spmv(A, ref.x))
        assert np.linalg.norm(xs - ref.x) <= (r * np.linalg.norm(b) + rr) / lam_min * (1 + 1e-6)


@pytest.mark.parametrize("nsys,lo,hi,seed,blocks,rows,gamma", [
    (5, 4, 24, 9, 0, 0, 1.0), (12, 8, 60, 10, 37, 64, 0.5), (12, 8, 60, 10, 7, 0, 1.5),
    (3, 2, 3, 11, 0, 32, 1.0)])
def test_batched_small(orc, nsys, lo, hi, seed, blocks, rows, gamma):
    spx = require_gpu()
    probs, bs = W.config4(nsys=nsys, lo=lo, hi=hi, seed=seed)
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    bvec = dev(np.concatenate(bs))
    x, iters, relres, st = batch.batch_cg(bvec, rtol=1e-8, blocks=blocks, rows_per_tile=rows,
                                          weight_exponent=gamma)
    assert st == 0
    check_systems(orc, probs, bs, host(x), iters, relres, 1e-8)


def test_batched_matches_single_solves():
    spx = require_gpu()
    probs, bs = W.config4(nsys=6, lo=10, hi=80, seed=12)
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    x, iters, relres, st = batch.batch_cg(dev(np.concatenate(bs)), rtol=1e-8)
    x = host(x)
    off = 0
    for m, b, it in zip(mats, bs, iters):
        r = m.cg_solve(dev(b), rtol=1e-8)
        assert abs(r.iters - it) <= 2
        xs = x[off:off + m.n]
        off += m.n
        assert np.linalg.norm(host(r.x) - xs) <= 1e-6 * np.linalg.norm(xs)


def test_batched_status_per_system():
    spx = require_gpu()
    good = W.five_point_system(6, np.ones(30), np.ones(30), np.ones(24))
    A = assemble(spx, good)
    Z = spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)), dev(np.array([1, 0, 1], np.int32)))
    Z.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    batch = spx.batch_create([A, Z])
    b = dev(np.ones(38))
    x, iters, relres, st = batch.batch_cg(b, rtol=1e-8)
    assert st == spx.ZERO_DIAGONAL
    assert relres[0] <= 1e-8 * 1.001
    # iteration limit
    batch2 = spx.batch_create([A])
    x, iters, relres, st = batch2.batch_cg(dev(np.ones(36)), rtol=1e-14, maxit=2)
    assert st == spx.NOT_CONVERGED and iters[0] == 2


@pytest.mark.parametrize("nsys,lo,hi,seed", [(40, 4, 40, 21), (7, 2, 70, 22), (1500, 3, 12, 23)])
def test_batched_persistent(orc, nsys, lo, hi, seed):
    """One launch for the whole batch, each workgroup solving whole systems
    from a queue (largest first): every system against its own oracle
    solve.  1500 systems exceed the resident workgroups, so workgroups take
    several systems each; the smallest systems are 3x3 grids."""
    spx = require_gpu()
    probs, bs = W.config4(nsys=nsys, lo=lo, hi=hi, seed=seed)
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    bvec = dev(np.concatenate(bs))
    x, iters, relres, st = batch.batch_cg(bvec, rtol=1e-8, persistent=1)
    assert st == 0
    check_systems(orc, probs, bs, host(x), iters, relres, 1e-8)
    # the launch-per-phase solve: the same iteration counts within 2, the
    # same solutions within the solves' tolerance
    x2, iters2, relres2, st2 = batch.batch_cg(bvec, rtol=1e-8, persistent=-1)
    assert st2 == 0
    assert max(abs(a - b) for a, b in zip(iters, iters2)) <= 2
    xh, x2h = host(x), host(x2)
    off = 0
    for p in probs:
        a, b2 = xh[off:off + p.n], x2h[off:off + p.n]
        off += p.n
        assert np.linalg.norm(a - b2) <= 1e-6 * np.linalg.norm(b2)


def test_batched_persistent_27_point_systems(orc):
    """3-D Q1 systems (27-entry rows, up to 13,824 rows, so 1024-thread
    workgroups with 256-row tiles) with log-normal coefficients, one
    persistent launch, every system against the oracle's CG."""
    spx = require_gpu()
    rng = np.random.default_rng(41)
    probs, bs = [], []
    for N in (2, 3, 5, 8, 11, 23):
        p = W.q1_poisson(N, 3, kappa=np.exp(rng.standard_normal(N**3)))
        probs.append(p)
        bs.append(rng.uniform(-1, 1, p.n))
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    x, iters, relres, st = batch.batch_cg(dev(np.concatenate(bs)), rtol=1e-9, persistent=1)
    assert st == 0
    xh = host(x)
    off = 0
    for s_, (p, b) in enumerate(zip(probs, bs)):
        A = orc.assemble(p.n, p.i, p.j, p.v)
        ref = orc.pcg(A, b, 1e-9)
        xs = xh[off:off + p.n]
        off += p.n
        assert ref.status == 0 and relres[s_] <= 1e-9 * (1 + 1e-3)
        assert np.linalg.norm(b - orc.spmv(A, xs)) <= 1e-9 * np.linalg.norm(b) * (1 + 1e-3)
        assert abs(iters[s_] - ref.iters) <= max(2, math.ceil(0.01 * ref.iters)), (s_, iters[s_], ref.iters)


def test_batched_persistent_statuses_and_guess():
    """A zero diagonal stops only its own system; the iteration limit; a
    second solve from the first one's solution stops at once."""
    spx = require_gpu()
    good = W.five_point_system(6, np.ones(30), np.ones(30), np.ones(24))
    A = assemble(spx, good)
    Z = spx.coo_preallocate(2, dev(np.array([0, 1, 1], np.int32)), dev(np.array([1, 0, 1], np.int32)))
    Z.set_values_coo(dev(np.array([1.0, 1.0, 2.0])))
    batch = spx.batch_create([A, Z, A])
    b = dev(np.ones(74))
    x, iters, relres, st = batch.batch_cg(b, rtol=1e-8, persistent=1)
    assert st == spx.ZERO_DIAGONAL
    assert relres[0] <= 1e-8 * 1.001 and relres[2] <= 1e-8 * 1.001 and iters[1] == 0
    x2, iters2, relres2, st2 = batch.batch_cg(b, x=x.clone(), rtol=1e-6, persistent=1)
    assert iters2[0] == 0 and iters2[2] == 0
    batch2 = spx.batch_create([A])
    x, iters, relres, st = batch2.batch_cg(dev(np.ones(36)), rtol=1e-14, maxit=2, persistent=1)
    assert st == spx.NOT_CONVERGED and iters[0] == 2


def test_batched_persistent_arguments():
    spx = require_gpu()
    A = assemble(spx, W.five_point_system(5, np.ones(20), np.ones(20), np.ones(20)))
    batch = spx.batch_create([A])
    with pytest.raises(spx.SpxError) as e:
        batch.batch_cg(dev(np.ones(25)), persistent=2)
    assert e.value.code == spx.INVALID_ARG
    # 256 dense rows: a 256-row tile of 65,536 entries does not fit
    n = 256
    i = np.repeat(np.arange(n, dtype=np.int32), n)
    j = np.tile(np.arange(n, dtype=np.int32), n)
    v = np.where(i == j, float(n), -1.0 / n)
    D = spx.coo_preallocate(n, dev(i), dev(j))
    D.set_values_coo(dev(v))
    batch = spx.batch_create([D])
    with pytest.raises(spx.SpxError) as e:
        batch.batch_cg(dev(np.ones(n)), persistent=1)
    assert e.value.code == spx.INVALID_ARG
    x, iters, relres, st = batch.batch_cg(dev(np.ones(n)), rtol=1e-10)
    assert st == 0 and relres[0] <= 1e-10 * 1.001


def test_autotune_takes_both_forms(orc):
    """The tuner times the persistent form beside launch shapes of the
    per-phase form and returns a working pick; on a batch the persistent
    form cannot take (a 256-row tile beyond its LDS) that candidate is
    skipped."""
    spx = require_gpu()
    probs, bs = W.config4(nsys=300, lo=4, hi=24, seed=31)
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    bvec = dev(np.concatenate(bs))
    cands = [autotune.Candidate(0, 0, 1.0, persistent=1), autotune.Candidate(1024, 0, 1.0),
             autotune.Candidate(2048, 64, 1.0)]
    best = autotune.tune_batch(batch, bvec, rtol=1e-8, candidates=cands)
    print("autotune:", best, flush=True)
    x, iters, relres, st = batch.batch_cg(bvec, rtol=1e-8, blocks=best["blocks"],
                                          rows_per_tile=best["rows_per_tile"],
                                          weight_exponent=best["weight_exponent"],
                                          persistent=best["persistent"])
    assert st == 0
    check_systems(orc, probs[:20], bs[:20], host(x)[:sum(p.n for p in probs[:20])], iters[:20],
                  relres[:20], 1e-8)
    n = 256
    i = np.repeat(np.arange(n, dtype=np.int32), n)
    j = np.tile(np.arange(n, dtype=np.int32), n)
    D = spx.coo_preallocate(n, dev(i), dev(j))
    D.set_values_coo(dev(np.where(i == j, float(n), -1.0 / n)))
    dense = spx.batch_create([D])
    best = autotune.tune_batch(dense, dev(np.ones(n)), rtol=1e-10, candidates=cands)
    assert best["persistent"] == -1


@pytest.mark.timeout(900)
def test_batched_full_config(orc):
    """The full 64-system batch (sides 32..512) to 1e-8, every system checked
    against its own oracle solve; also the autotuner's pick."""
    spx = require_gpu()
    probs, bs = W.config4()
    print("batch sizes:", [p.grid for p in probs], flush=True)
    mats = [assemble(spx, p) for p in probs]
    batch = spx.batch_create(mats)
    bvec = dev(np.concatenate(bs))
    x, iters, relres, st = batch.batch_cg(bvec, rtol=1e-8)
    assert st == 0
    print("iterations:", iters, flush=True)
    check_systems(orc, probs, bs, host(x), iters, relres, 1e-8)
    best = autotune.tune_batch(batch, bvec, rtol=1e-8,
                               candidates=[autotune.Candidate(1024, 0, 1.0),
                                           autotune.Candidate(2048, 64, 1.0)])
    print("autotune:", best, flush=True)
    x2, iters2, relres2, st2 = batch.batch_cg(bvec, rtol=1e-8, blocks=best["blocks"],
                                              rows_per_tile=best["rows_per_tile"],
                                              weight_exponent=best["weight_exponent"],
                                              persistent=best["persistent"])
    assert st2 == 0 and max(relres2) <= 1e-8 * 1.001


def test_spmm_full_size_sampled(orc):
    spx = require_gpu()
    prob, _, _ = W.config2(127)
    A = assemble(spx, prob)
    X = W.spmm_rhs(prob.n, 16)
    Y = host(A.spmm(dev(X)))
    rows = np.unique(np.random.default_rng(5).integers(0, prob.n, 500)).astype(np.int32)
    ptr, scol, sval = orc.coo_rows(prob.n, prob.i, prob.j, prob.v, rows)
    for s, r in enumerate(rows):
        c, v = scol[ptr[s]:ptr[s + 1]], sval[ptr[s]:ptr[s + 1]]
        ref = np.zeros(16)
        for cc, vv in zip(c, v):
            ref += vv * X[cc]
        scale = np.abs(v) @ np.abs(X[c])
        assert np.all(np.abs(Y[r] - ref) <= 1e-12 * scale + 1e-300)


def test_batched_with_a_system_without_window(orc):
    """One system's random pattern has no window index, so the whole batch
    takes the stream walk; every system still converges and matches its
    single-system solve."""
    spx = require_gpu()
    probs, bs = W.config4(nsys=4, lo=20, hi=90, seed=13)
    rng = np.random.default_rng(14)
    n = 9000
    i = rng.integers(0, n, 60000).astype(np.int32)
    j = rng.integers(0, n, 60000).astype(np.int32)
    v = rng.uniform(-1, 1, i.size)
    diag = 1.0 + np.bincount(i, np.abs(v), n) + np.bincount(j, np.abs(v), n)
    k = np.arange(n, dtype=np.int32)
    rand = W.CooProblem(n=n, i=np.concatenate([i, j, k]), j=np.concatenate([j, i, k]),
                        v=np.concatenate([v, v, diag]))
    mats = [assemble(spx, p) for p in probs] + [assemble(spx, rand)]
    assert all(m.get_window(arrays=False)["built"] for m in mats[:-1])
    assert not mats[-1].get_window(arrays=False)["built"]
    b_r = rng.uniform(-1, 1, n)
    allb = bs + [b_r]
    batch = spx.batch_create(mats)
    x, iters, relres, st = batch.batch_cg(dev(np.concatenate(allb)), rtol=1e-9)
    assert st == 0 and max(relres) <= 1e-9 * 1.001
    x = host(x)
    off = 0
    for m, b, it in zip(mats, allb, iters):
        r = m.cg_solve(dev(b), rtol=1e-9)
        assert abs(r.iters - it) <= 2
        xs = x[off:off + m.n]
        off += m.n
        assert np.linalg.norm(host(r.x) - xs) <= 1e-6 * np.linalg.norm(xs)
