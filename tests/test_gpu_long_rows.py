"""Solvers on a matrix with one very long row and column (an arrow).  At
20000 rows no row tile fits in LDS, so every solver form falls back to the
lane walk and the one-workgroup solve declines; at 1500 rows the
one-workgroup solve runs with the long row inside one of its tiles."""
import math

import numpy as np
import pytest

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def arrow(n, seed, nonsym=False):
    """An arrow on a band.  Rows 1..n-1 form a tridiagonal band with
    diagonal 2.5 + U[0, 1) and off-diagonals -1 (-1.3 below, -0.7 above when
    non-symmetric); row and column 0 are dense with entries of size up to
    1/sqrt(n), and a_00 = 1 + the sum of their magnitudes.  By Gershgorin the
    symmetric part has every eigenvalue >= 0.5 - 1/sqrt(n)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, n - 1) / math.sqrt(n)
    w = rng.uniform(-1, 1, n - 1) / math.sqrt(n) if nonsym else u
    d = 2.5 + rng.uniform(0, 1, n)
    d[0] = 1.0 + 0.5 * (np.abs(u).sum() + np.abs(w).sum())
    lo, hi = (-1.3, -0.7) if nonsym else (-1.0, -1.0)
    r = np.arange(1, n, dtype=np.int32)
    band = np.arange(1, n - 1, dtype=np.int32)
    i = np.concatenate([np.arange(n, dtype=np.int32), np.zeros(n - 1, np.int32), r, band + 1, band])
    j = np.concatenate([np.arange(n, dtype=np.int32), r, np.zeros(n - 1, np.int32), band, band + 1])
    v = np.concatenate([d, u, w, np.full(n - 2, lo), np.full(n - 2, hi)])
    return W.CooProblem(n=n, i=i, j=j, v=v), rng.uniform(-1, 1, n)


LAM_MIN = 0.45  # below 0.5 - 1/sqrt(n) for every n used here


@pytest.mark.parametrize("n", [1500, 20000])
def test_arrow_cg_forms(orc, n):
    spx = require_gpu()
    prob, b = arrow(n, 70)
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    ores = orc.pcg(ref, b, 1e-10)
    for variant, small in ((0, 1), (1, 1), (0, 2)):
        A.set_option(spx.OPT_CG_VARIANT, variant)
        A.set_option(spx.OPT_SMALL_SOLVE, small)
        res = A.cg_solve(dev(b), rtol=1e-10)
        assert res.status == 0 and ores.status == 0
        assert res.relres <= 1e-10 * (1 + 1e-3)
        assert abs(res.iters - ores.iters) <= max(2, math.ceil(0.01 * ores.iters))
        x = host(res.x)
        r_gpu = np.linalg.norm(b - orc.spmv(ref, x))
        r_ref = np.linalg.norm(b - orc.spmv(ref, ores.x))
        assert np.linalg.norm(x - ores.x) <= (r_gpu + r_ref) / LAM_MIN * (1 + 1e-6)
    A.set_option(spx.OPT_CG_VARIANT, 0)
    m = A.cg_solve_mixed(dev(b), rtol_outer=1e-10, rtol_inner=1e-4)
    assert m.status == 0 and m.relres <= 1e-10


def test_arrow_in_batches(orc):
    spx = require_gpu()
    prob, b = arrow(6000, 71)
    five = W.five_point_system(8, np.ones(56), np.ones(56), np.ones(32))
    b5 = np.random.default_rng(72).uniform(-1, 1, five.n)
    batch = spx.batch_create([assemble(spx, prob), assemble(spx, five)])
    bvec = dev(np.concatenate([b, b5]))
    x, iters, relres, st = batch.batch_cg(bvec, rtol=1e-9)
    assert st == 0 and max(relres) <= 1e-9 * 1.001
    xs = host(x)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    assert np.linalg.norm(b - orc.spmv(ref, xs[:prob.n])) <= 1e-9 * np.linalg.norm(b) * 1.001
    nprob, nb = arrow(6000, 73, nonsym=True)
    nbatch = spx.batch_create([assemble(spx, nprob), assemble(spx, five)])
    nvec = dev(np.concatenate([nb, b5]))
    nref = orc.assemble(nprob.n, nprob.i, nprob.j, nprob.v)
    for fn in (nbatch.batch_bicg, nbatch.batch_tfqmr):
        x, iters, relres, st = fn(nvec, rtol=1e-9)
        assert st == 0 and max(relres) <= 1e-9 * 1.001
        xs = host(x)
        assert np.linalg.norm(nb - orc.spmv(nref, xs[:nprob.n])) <= 1e-9 * np.linalg.norm(nb) * 1.001
