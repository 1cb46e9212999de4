"""Window walk of the products: the device-built window index against a
numpy construction from its definition, and products and solves taken
through it, which must be bitwise those of the oracle and of the stream
walk (the window walk changes where x is read from, not the arithmetic)."""
import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, bits, dev, host, require_gpu

pytestmark = pytest.mark.gpu

ROWS, BLOCK, MAX_BLOCKS, SPAN = 256, 64, 64, 8192


def window_reference(rowptr, col, n):
    """Per tile of 256 rows: the ascending distinct blocks col // 64 of its
    entries, or no window when they span 8192 blocks or more or number more
    than 64; lcol = rank of the block * 64 + col % 64.  The index is kept when
    windows hold at most two x entries per matrix entry and at most one entry
    in eight sits in a tile without a window."""
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    tiles = (n + ROWS - 1) // ROWS
    ptr, blk, gather, biggest = [0], [], 0, 0
    lcol = np.full(col.size, -1, np.int64)
    for t in range(tiles):
        a, b = rowptr[t * ROWS], rowptr[min(n, (t + 1) * ROWS)]
        if b > a:
            bl = col[a:b] // BLOCK
            u = np.unique(bl)
            if bl.max() - bl.min() < SPAN and u.size <= MAX_BLOCKS:
                blk.extend(u.tolist())
                lcol[a:b] = np.searchsorted(u, bl) * BLOCK + col[a:b] % BLOCK
                biggest = max(biggest, u.size)
            else:
                gather += b - a
        ptr.append(len(blk))
    nnz = col.size
    built = biggest > 0 and len(blk) * BLOCK <= 2 * nnz and 8 * gather <= nnz
    return dict(built=built, ptr=np.array(ptr), blk=np.array(blk, np.int64), lcol=lcol,
                gather=gather, biggest=biggest)


def spiked(seed):
    """3-D Q1 operator (31^3 nodes) with one row given 2000 extra entries
    spread over all columns (its tile reads x directly) and the rows of one
    whole 256-row tile removed (an empty tile)."""
    prob = W.q1_poisson(30, 3, kappa=np.exp(np.random.default_rng(seed).standard_normal(30**3)))
    rng = np.random.default_rng(seed + 1)
    keep = ~((prob.i >= 512) & (prob.i < 768))
    extra_j = rng.integers(0, prob.n, 2000).astype(np.int32)
    i = np.concatenate([prob.i[keep], np.full(2000, 3000, np.int32)])
    j = np.concatenate([prob.j[keep], extra_j])
    v = np.concatenate([prob.v[keep], rng.uniform(-1, 1, 2000)])
    return W.CooProblem(n=prob.n, i=i, j=j, v=v)


def banded_arrays(n, half, seed):
    p = banded(n, half, seed)
    return p.i, p.j, p.v


def banded(n, half, seed):
    rng = np.random.default_rng(seed)
    i, j = [], []
    for d in range(-half, half + 1):
        r = np.arange(max(0, -d), min(n, n - d))
        i.append(r)
        j.append(r + d)
    i = np.concatenate(i).astype(np.int32)
    j = np.concatenate(j).astype(np.int32)
    v = rng.uniform(-1, 1, i.size) + np.where(i == j, 2.0 * half + 2.0, 0.0)
    return W.CooProblem(n=n, i=i, j=j, v=v)


def make(case):
    if case == "q1_3d":
        return W.q1_poisson(24, 3, kappa=np.exp(np.random.default_rng(80).standard_normal(24**3)))
    if case == "q1_2d":
        return W.q1_poisson(100, 2)
    if case == "spiked":
        return spiked(81)
    if case == "n257":
        return banded(257, 3, 82)
    if case == "n7":
        return banded(7, 6, 83)
    raise ValueError(case)


CASES = ["q1_3d", "q1_2d", "spiked", "n257", "n7"]


@pytest.mark.parametrize("case", CASES)
def test_window_index_matches_definition(orc, case):
    spx = require_gpu()
    prob = make(case)
    A = assemble(spx, prob)
    ref_A = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    for transpose in (False, True):
        rowptr, col, _ = A.get_csr(transpose)
        ref = window_reference(host(rowptr), host(col), prob.n)
        w = A.get_window(transpose)
        assert w["built"] == ref["built"], (case, transpose, w, ref["gather"], ref["biggest"])
        if not ref["built"]:
            continue
        assert w["max_blocks"] == ref["biggest"] and w["gather_entries"] == ref["gather"]
        assert w["total_blocks"] == ref["blk"].size
        assert np.array_equal(host(w["ptr"]), ref["ptr"])
        assert np.array_equal(host(w["blk"]), ref["blk"])
        lcol = host(w["lcol"]).astype(np.int64)
        mask = ref["lcol"] >= 0
        assert np.array_equal(lcol[mask], ref["lcol"][mask])
    if case in ("q1_3d", "q1_2d", "spiked"):
        assert A.get_window()["built"]
        A.set_option(spx.OPT_SPMV_VARIANT, 4)
        assert A.get_option(spx.OPT_SPMV_VARIANT) == 4
    if case == "spiked":
        assert A.get_window()["gather_entries"] > 2000
    del ref_A


@pytest.mark.parametrize("case", CASES)
def test_window_products_bitwise(orc, case):
    spx = require_gpu()
    prob = make(case)
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SPMV_VARIANT, 4)
    assert A.get_option(spx.OPT_SPMV_VARIANT) == 4
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    rng = np.random.default_rng(90)
    x = rng.uniform(-1, 1, prob.n)
    y_ref = bits(orc.spmv(ref, x))
    yt_ref = bits(orc.spmv_transpose(ref, x))
    xd = dev(x)
    # the same x at an address that is 8 but not 16 bytes aligned
    buf = torch.zeros(prob.n + 1, dtype=torch.float64, device="cuda")
    buf[1:] = xd
    xu = buf[1:]
    assert xu.data_ptr() % 16 == 8
    for nt in (1, 0):
        for remap in (1, 0):
            A.set_option(spx.OPT_NONTEMPORAL, nt)
            A.set_option(spx.OPT_XCD_REMAP, remap)
            assert np.array_equal(bits(host(A.matmult(xd))), y_ref)
            assert np.array_equal(bits(host(A.matmult(xu))), y_ref)
            assert np.array_equal(bits(host(A.matmult_transpose(xd))), yt_ref)
            assert np.array_equal(bits(host(A.matmult_transpose(xu))), yt_ref)


@pytest.mark.parametrize("remap", [1, 0])
def test_window_solvers_match_stream_walk(remap):
    """With the same solver grid, block order and tiles of the same 256 rows,
    the window walk and the stream walk give every workgroup the same rows and
    the same row sums, so every solver form takes the same iterates: same
    iteration counts, bitwise the same solutions.  (Another grid, order or
    tile size moves rows between workgroups and changes the rounding of the
    dot products, not the products.)"""
    spx = require_gpu()
    prob = make("q1_3d")
    b = dev(np.random.default_rng(91).uniform(-1, 1, prob.n))
    out = {}
    for variant in (4, 2):
        A = assemble(spx, prob)
        A.set_option(spx.OPT_SPMV_VARIANT, variant)
        A.set_option(spx.OPT_SOLVER_BLOCKS, 48)
        A.set_option(spx.OPT_XCD_REMAP, remap)
        if variant == 2:
            A.set_option(spx.OPT_ROWS_PER_BLOCK, 256)
            A.set_option(spx.OPT_ROWS_PER_BLOCK_F32, 256)
        assert A.get_option(spx.OPT_SPMV_VARIANT) == variant
        assert A.get_option(spx.OPT_ROWS_PER_BLOCK) == 256
        assert A.get_option(spx.OPT_XCD_REMAP) == remap
        r = A.cg_solve(b, rtol=1e-10)
        A.set_option(spx.OPT_CG_VARIANT, 1)
        sr = A.cg_solve(b, rtol=1e-10)
        A.set_option(spx.OPT_CG_VARIANT, 0)
        m = A.cg_solve_mixed(b, rtol_outer=1e-10, rtol_inner=1e-4)
        t = A.cg_solve_transpose(b, rtol=1e-10)
        out[variant] = [(r.iters, host(r.x)), (sr.iters, host(sr.x)), (m.inner, host(m.x)),
                        (t.iters, host(t.x))]
        assert r.status == 0 and sr.status == 0 and m.status == 0 and t.status == 0
    for (i0, x0), (i2, x2) in zip(out[4], out[2]):
        assert i0 == i2 and np.array_equal(bits(x0), bits(x2))


def test_window_option_resolution(orc):
    spx = require_gpu()
    # a random pattern gets no index: asking for the window walk gives the
    # automatic choice
    rng = np.random.default_rng(92)
    prob = W.random_coo(rng, 9000, 120000, extreme=False)
    A = assemble(spx, prob)
    assert not A.get_window()["built"]
    auto = A.get_option(spx.OPT_SPMV_VARIANT)
    A.set_option(spx.OPT_SPMV_VARIANT, 4)
    assert A.get_option(spx.OPT_SPMV_VARIANT) == auto
    # a small system: auto keeps the stream walk, the window walk on request
    B = assemble(spx, make("q1_3d"))
    assert B.get_window()["built"] and B.get_option(spx.OPT_SPMV_VARIANT) == 2
    B.set_option(spx.OPT_SPMV_VARIANT, 4)
    assert B.get_option(spx.OPT_SPMV_VARIANT) == 4
    B.set_option(spx.OPT_SPMV_VARIANT, 1)
    assert B.get_option(spx.OPT_SPMV_VARIANT) == 1
    # a large one (12 or more 256-row tiles per compute unit): auto takes the
    # window walk, and options of the stream walk keep the stream walk
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    C = assemble(spx, banded(12 * 256 * cus + 5, 3, 93))
    assert C.get_window()["built"] and C.get_option(spx.OPT_SPMV_VARIANT) == 4
    C.set_option(spx.OPT_ROWS_PER_BLOCK, 64)
    assert C.get_option(spx.OPT_SPMV_VARIANT) == 2
    C.set_option(spx.OPT_ROWS_PER_BLOCK, 0)
    C.set_option(spx.OPT_QUAD_LOADS, 1)
    assert C.get_option(spx.OPT_SPMV_VARIANT) == 2
    C.set_option(spx.OPT_QUAD_LOADS, 0)
    assert C.get_option(spx.OPT_SPMV_VARIANT) == 4
    # block order by default: plain for the window walk, XCD order otherwise;
    # an explicit order holds for every walk, -1 restores the choice
    assert C.get_option(spx.OPT_XCD_REMAP) == 0
    assert B.get_option(spx.OPT_XCD_REMAP) == 1
    C.set_option(spx.OPT_XCD_REMAP, 1)
    assert C.get_option(spx.OPT_XCD_REMAP) == 1
    y1 = host(C.matmult(dev(np.random.default_rng(94).uniform(-1, 1, C.n))))
    C.set_option(spx.OPT_XCD_REMAP, -1)
    assert C.get_option(spx.OPT_XCD_REMAP) == 0
    ref = orc.assemble(C.n, *banded_arrays(12 * 256 * cus + 5, 3, 93))
    x = np.random.default_rng(94).uniform(-1, 1, C.n)
    assert np.array_equal(bits(host(C.matmult(dev(x)))), bits(orc.spmv(ref, x)))
    assert np.array_equal(bits(y1), bits(orc.spmv(ref, x)))
    with pytest.raises(spx.SpxError):
        B.set_option(spx.OPT_SPMV_VARIANT, 5)


def test_matmult_window_threshold(orc):
    """MatMult takes the window walk from 2.5 tiles of 256 rows per compute
    unit (its loads go out together), the solvers from 12: on the 3-D Q1
    operator with 58^3 nodes (about 3 tiles per CU on 256 CUs) MatMult
    reports and runs the window walk, bitwise the oracle's product and
    transposed product, and CG on the solvers' own walk still matches the
    oracle's residual bound."""
    spx = require_gpu()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    N = 57
    prob = W.q1_poisson(N, 3)
    n = prob.n
    tiles = (n + 255) // 256
    assert 2.5 * cus <= tiles < 12 * cus
    A = assemble(spx, prob)
    assert A.get_window()["built"] and A.get_option(spx.OPT_SPMV_VARIANT) == 4
    ref = orc.assemble(n, prob.i, prob.j, prob.v)
    x = np.random.default_rng(97).uniform(-1, 1, n)
    assert np.array_equal(bits(host(A.matmult(dev(x)))), bits(orc.spmv(ref, x)))
    refT = orc.assemble(n, prob.j, prob.i, prob.v)
    assert np.array_equal(bits(host(A.matmult_transpose(dev(x)))), bits(orc.spmv(refT, x)))
    b_h = np.random.default_rng(98).uniform(-1, 1, n)
    r = A.cg_solve(dev(b_h), rtol=1e-10)
    assert r.status == 0
    res = b_h - orc.spmv(ref, host(r.x))
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(b_h)
    # half as many tiles: MatMult keeps the stream walk
    small = assemble(spx, W.q1_poisson(45, 3))
    if (small.n + 255) // 256 < 2.5 * cus:
        assert small.get_option(spx.OPT_SPMV_VARIANT) != 4


def stencil_problem(shape, offsets, seed):
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    I, J = [], []
    for off in offsets:
        src = idx[tuple(slice(max(0, -o), s - max(0, o)) for o, s in zip(off, shape))]
        dst = idx[tuple(slice(max(0, o), s - max(0, -o)) for o, s in zip(off, shape))]
        I.append(src.ravel())
        J.append(dst.ravel())
    i = np.concatenate(I).astype(np.int32)
    j = np.concatenate(J).astype(np.int32)
    v = np.random.default_rng(seed).uniform(-1, 1, i.size)
    return W.CooProblem(n=n, i=i, j=j, v=v)


SHAPES = {
    "band1": lambda: banded(3001, 1, 95),
    "band20": lambda: banded(4999, 20, 96),
    "band900": lambda: banded(6000, 900, 97),  # windows near or over the 64-block limit
    "5pt_2d": lambda: stencil_problem((77, 61), [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)], 98),
    "7pt_3d": lambda: stencil_problem((17, 13, 11), [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0),
                                                      (0, -1, 0), (0, 0, 1), (0, 0, -1)], 99),
    "9pt_2d": lambda: stencil_problem((90, 45), [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)], 100),
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_window_other_patterns(orc, name):
    """The index against its definition and the window-walk products bitwise
    against the oracle on banded matrices (up to half-width 900) and 5-, 7-
    and 9-point stencils on ragged grids."""
    spx = require_gpu()
    prob = SHAPES[name]()
    A = assemble(spx, prob)
    rowptr, col, _ = A.get_csr()
    ref = window_reference(host(rowptr), host(col), prob.n)
    w = A.get_window()
    assert w["built"] == ref["built"]
    if w["built"]:
        assert np.array_equal(host(w["ptr"]), ref["ptr"])
        assert np.array_equal(host(w["blk"]), ref["blk"])
        mask = ref["lcol"] >= 0
        assert np.array_equal(host(w["lcol"]).astype(np.int64)[mask], ref["lcol"][mask])
        A.set_option(spx.OPT_SPMV_VARIANT, 4)
        assert A.get_option(spx.OPT_SPMV_VARIANT) == 4
    oref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    x = np.random.default_rng(101).uniform(-1, 1, prob.n)
    assert np.array_equal(bits(host(A.matmult(dev(x)))), bits(orc.spmv(oref, x)))
    assert np.array_equal(bits(host(A.matmult_transpose(dev(x)))), bits(orc.spmv_transpose(oref, x)))
