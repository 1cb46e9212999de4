"""Diagonal / off-diagonal split of one rank's rows (paper Sec. 5) against
the oracle.

The expected blocks are built here from the definition: a kept triplet with
its row in [lo, hi) belongs to the diagonal block when its column is in
[lo, hi) too (local numbers), else to the off-diagonal block, whose rows are
the local rows with an off-diagonal entry and whose columns are the distinct
off-diagonal global columns, both ascending; every other triplet gets index
-1 in that block's stream.  The oracle assembles each stream; the GPU blocks
must equal them bitwise (pattern, values, maps).  The split product must
match the oracle's product of the whole slab (rows [lo, hi), every column)
within 1e-12 componentwise.
"""
import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def expected_streams(prob, lo, hi):
    i = prob.i.astype(np.int64)
    j = prob.j.astype(np.int64)
    kept = (i >= 0) & (j >= 0)
    mine = kept & (i >= lo) & (i < hi)
    diag = mine & (j >= lo) & (j < hi)
    off = mine & ~diag
    garray = np.unique(j[off]).astype(np.int32)
    orows = np.unique(i[off] - lo).astype(np.int32)
    i_d = np.where(diag, i - lo, -1).astype(np.int32)
    j_d = np.where(diag, j - lo, -1).astype(np.int32)
    i_o = np.where(off, np.searchsorted(orows, i - lo), -1).astype(np.int32)
    j_o = np.where(off, np.searchsorted(garray, j), -1).astype(np.int32)
    nremote = int(np.sum(kept & ~mine))
    return (i_d, j_d), (i_o, j_o), garray, orows, nremote


def check_split(spx, orc, prob, lo, hi, x_global, seed=0):
    n = prob.n
    S = spx.split_preallocate(n, lo, hi, dev(prob.i), dev(prob.j))
    S.set_values_coo(dev(prob.v))
    (i_d, j_d), (i_o, j_o), garray, orows, nremote = expected_streams(prob, lo, hi)
    m = hi - lo
    assert (S.rows, S.nghost, S.nrows_offdiag, S.nremote) == (m, len(garray), len(orows), nremote)
    g, o = (host(t) for t in S.maps())
    assert np.array_equal(g, garray) and np.array_equal(o, orows)
    no = max(len(orows), len(garray), 1)
    for blk, (ii, jj, order) in ((S.diag, (i_d, j_d, m)), (S.offdiag, (i_o, j_o, no))):
        ref = orc.assemble(order, ii, jj, prob.v)
        rowptr, col, val = (host(t) for t in blk.get_csr())
        assert np.array_equal(rowptr, ref.rowptr) and np.array_equal(col, ref.col)
        assert np.array_equal(bits(val), bits(ref.val))
        jm, pm = (host(t) for t in blk.get_coo_maps())
        assert np.array_equal(jm.astype(np.int64), ref.jmap) and np.array_equal(pm, ref.perm)
    # the product against the oracle's product of the whole slab
    xg_d = dev(x_global)
    x_ghost = S.gather_ghosts(xg_d)
    assert np.array_equal(bits(host(x_ghost)), bits(x_global[garray]))
    y = host(S.matmult(dev(x_global[lo:hi]), x_ghost))
    i_s = np.where((prob.i >= lo) & (prob.i < hi), prob.i, -1).astype(np.int32)
    slab = orc.assemble(n, i_s, prob.j, prob.v)
    y_ref = orc.spmv(slab, x_global)[lo:hi]
    scale = orc.abs_spmv(slab, x_global)[lo:hi]
    bad = np.flatnonzero(np.abs(y - y_ref) > 1e-12 * scale + 1e-300)
    assert bad.size == 0, (bad[:5], y[bad[:5]], y_ref[bad[:5]])
    # ADD mode adds the same sums again to both blocks
    S.set_values_coo(dev(prob.v), mode=spx.ADD_VALUES)
    for blk, (ii, jj, order) in ((S.diag, (i_d, j_d, m)), (S.offdiag, (i_o, j_o, no))):
        ref = orc.assemble(order, ii, jj, prob.v)
        val = host(blk.get_csr()[2])
        assert np.array_equal(bits(val), bits(ref.val + ref.val))
    S.destroy()
    return len(garray), len(orows), nremote


@pytest.mark.parametrize("lo,hi", [(0, 57), (57, 171), (171, 300), (0, 300), (120, 121)])
def test_split_random_stream(orc, lo, hi):
    """Non-symmetric fuzz stream: duplicates, negative indices, +-0.0,
    magnitudes 2^+-60; slabs at either end, in the middle, the whole matrix
    (no off-diagonal block) and a single row."""
    spx = require_gpu()
    rng = np.random.default_rng(11)
    prob = W.random_coo(rng, 300, 20000)
    x = rng.uniform(-1, 1, prob.n)
    ng, nro, nrem = check_split(spx, orc, prob, lo, hi, x)
    if (lo, hi) == (0, 300):
        assert ng == 0 and nro == 0 and nrem == 0


def test_split_block_diagonal_has_no_ghosts(orc):
    """Two decoupled 2-D grids stacked: the slab that is one grid has an
    empty off-diagonal block."""
    spx = require_gpu()
    a = W.q1_poisson(9, 2)
    b = W.q1_poisson(7, 2)
    prob = W.CooProblem(n=a.n + b.n, i=np.concatenate([a.i, b.i + a.n]).astype(np.int32),
                        j=np.concatenate([a.j, b.j + a.n]).astype(np.int32),
                        v=np.concatenate([a.v, b.v]))
    x = np.random.default_rng(3).uniform(-1, 1, prob.n)
    ng, nro, nrem = check_split(spx, orc, prob, 0, a.n, x)
    assert ng == 0 and nro == 0 and nrem == b.i.size


@pytest.mark.parametrize("N,slabs,which", [(12, 4, 1), (12, 4, 0), (12, 4, 3), (31, 8, 5)])
def test_split_q1_slabs(orc, N, slabs, which):
    """Row slabs of the 3-D Q1 operator (z planes split evenly): the ghosts
    are the planes just below and above the slab."""
    spx = require_gpu()
    prob = W.q1_poisson(N, 3, kappa=np.exp(np.random.default_rng(N).standard_normal(N**3)))
    M = N + 1
    planes = np.linspace(0, M, slabs + 1).astype(int)
    lo, hi = planes[which] * M * M, planes[which + 1] * M * M
    x = np.random.default_rng(5).uniform(-1, 1, prob.n)
    ng, nro, _ = check_split(spx, orc, prob, lo, hi, x)
    expect = (M * M) * ((which > 0) + (which < slabs - 1))
    assert ng == expect and nro == expect


def test_split_full_size_slab(orc):
    """One GPU's share of an 8-way slab partition of the 128^3-node
    workload: 16 planes of 128^2 rows, ghosts two planes."""
    spx = require_gpu()
    prob, x, _ = W.config2(127)
    plane = 128 * 128
    lo, hi = 48 * plane, 64 * plane
    ng, nro, nrem = check_split(spx, orc, prob, lo, hi, x)
    assert ng == 2 * plane and nro == 2 * plane
    print(f"[split] full-size slab: {hi - lo} rows, {ng} ghosts, {nro} off-diagonal rows, "
          f"{nrem} remote triplets", flush=True)


def test_split_errors():
    spx = require_gpu()
    i = dev(np.array([0, 1, 2], np.int32))
    j = dev(np.array([0, 5, 1], np.int32))
    with pytest.raises(spx.SpxError) as e:
        spx.split_preallocate(3, 0, 2, i, j)
    assert e.value.code == spx.INDEX_OUT_OF_RANGE
    for lo, hi in ((1, 1), (2, 1), (-1, 2), (0, 4)):
        with pytest.raises(spx.SpxError) as e:
            spx.split_preallocate(3, lo, hi, i, dev(np.array([0, 1, 2], np.int32)))
        assert e.value.code == spx.INVALID_ARG
