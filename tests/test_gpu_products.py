"""GPU products (MatMult, MatMultTranspose, SpMM, SDDMM, COO gather) against
the oracle."""
import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import assemble, bits, dev, host, require_gpu, spmv_within

pytestmark = pytest.mark.gpu


def test_config1_matmult(orc):
    spx = require_gpu()
    prob, x, _ = W.config1()
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    y = host(A.matmult(dev(x)))
    spmv_within(y, orc.spmv(ref, x), orc.abs_spmv(ref, x))
    yt = host(A.matmult_transpose(dev(x)))
    spmv_within(yt, orc.spmv_transpose(ref, x), orc.abs_spmv_transpose(ref, x))


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_matmult_every_lane_count(orc, lanes):
    spx = require_gpu()
    rng = np.random.default_rng(20 + lanes)
    prob = W.random_coo(rng, 3001, 150000, extreme=False)
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SPMV_LANES, lanes)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    x = rng.uniform(-1, 1, prob.n)
    y = host(A.matmult(dev(x)))
    spmv_within(y, orc.spmv(ref, x), orc.abs_spmv(ref, x))
    yt = host(A.matmult_transpose(dev(x)))
    spmv_within(yt, orc.spmv_transpose(ref, x), orc.abs_spmv_transpose(ref, x))
    # the block order does not change any row's arithmetic
    A.set_option(spx.OPT_XCD_REMAP, 0)
    y2 = host(A.matmult(dev(x)))
    assert np.array_equal(bits(y), bits(y2))


@pytest.mark.parametrize("variant,rows", [(1, 0), (2, 32), (2, 64), (2, 128), (2, 256), (3, 0),
                                          (3, 32), (3, 64), (4, 0)])
@pytest.mark.parametrize("case", ["q1_3d", "random", "config1"])
def test_matmult_variants(orc, variant, rows, case):
    spx = require_gpu()
    rng = np.random.default_rng(7)
    if case == "q1_3d":
        prob = W.q1_poisson(20, 3, kappa=np.exp(rng.standard_normal(20**3)))
    elif case == "random":
        prob = W.random_coo(rng, 7001, 90000, extreme=False)
    else:
        prob = W.config1()[0]
    A = assemble(spx, prob)
    A.set_option(spx.OPT_SPMV_VARIANT, variant)
    A.set_option(spx.OPT_ROWS_PER_BLOCK, rows)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    x = rng.uniform(-1, 1, prob.n)
    y = host(A.matmult(dev(x)))
    yr = orc.spmv(ref, x)
    spmv_within(y, yr, orc.abs_spmv(ref, x))
    if variant >= 2 and A.get_option(spx.OPT_SPMV_VARIANT) == variant:
        # products rounded then added in row order: the oracle's arithmetic
        assert np.array_equal(bits(y), bits(yr))
    yt = host(A.matmult_transpose(dev(x)))
    spmv_within(yt, orc.spmv_transpose(ref, x), orc.abs_spmv_transpose(ref, x))
    for nt in (0, 1):
        for quad in (0, 1):
            A.set_option(spx.OPT_NONTEMPORAL, nt)
            A.set_option(spx.OPT_QUAD_LOADS, quad)
            assert np.array_equal(bits(host(A.matmult(dev(x)))), bits(y))


def test_matmult_long_and_empty_rows(orc):
    spx = require_gpu()
    rng = np.random.default_rng(30)
    n = 5000
    # one very long row, many empty rows, a dense column
    i = np.concatenate([np.zeros(40000, np.int32), rng.integers(0, n // 2, 20000).astype(np.int32),
                        rng.integers(0, n, 3000).astype(np.int32)])
    j = np.concatenate([rng.integers(0, n, 40000).astype(np.int32),
                        rng.integers(0, n // 2, 20000).astype(np.int32), np.full(3000, 7, np.int32)])
    v = rng.uniform(-1, 1, i.size)
    prob = W.CooProblem(n=n, i=i, j=j, v=v)
    A = assemble(spx, prob)
    ref = orc.assemble(n, i, j, v)
    x = rng.uniform(-1, 1, n)
    spmv_within(host(A.matmult(dev(x))), orc.spmv(ref, x), orc.abs_spmv(ref, x))
    spmv_within(host(A.matmult_transpose(dev(x))), orc.spmv_transpose(ref, x),
                orc.abs_spmv_transpose(ref, x))


def test_matmult_deterministic_and_transpose_identity(orc):
    spx = require_gpu()
    rng = np.random.default_rng(31)
    prob = W.random_coo(rng, 20000, 400000, extreme=False)
    A = assemble(spx, prob)
    x, z = (dev(rng.uniform(-1, 1, prob.n)) for _ in range(2))
    y0 = host(A.matmult(x))
    for _ in range(5):
        assert np.array_equal(bits(host(A.matmult(x))), bits(y0))
    lhs = float(torch.dot(z, A.matmult(x)))
    rhs = float(torch.dot(A.matmult_transpose(z), x))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)) * 100


def test_spmm_matches_oracle(orc):
    spx = require_gpu()
    prob, _, _ = W.config1()
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    for nrhs in (1, 3, 16, 40):
        X = W.spmm_rhs(prob.n, nrhs)
        Y = host(A.spmm(dev(X)))
        Yr = orc.spmm(ref, X)
        for c in range(nrhs):
            spmv_within(Y[:, c], Yr[:, c], orc.abs_spmv(ref, X[:, c]))


def test_spmm_layouts_bitwise(orc):
    """Through the C ABI with explicit leading dimensions: the paired-column
    kernel (16-byte aligned X and Y, even ld; an odd last column on its own)
    and the one-column-per-lane kernel (8-byte aligned X) give the same bits,
    within the SpMV tolerance of the oracle."""
    import ctypes
    spx = require_gpu()
    lib = spx.load_library()
    rng = np.random.default_rng(34)
    prob = W.random_coo(rng, 5003, 90000, extreme=False)
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    n = prob.n
    for nrhs in (1, 7, 16):
        Xh = rng.uniform(-1, 1, (n, nrhs))
        ld = nrhs + 1 if nrhs % 2 else nrhs + 2  # even, padded rows
        Xa = torch.zeros(n * ld + 2, dtype=torch.float64, device="cuda")
        Xa[: n * ld].view(n, ld)[:, :nrhs] = dev(Xh)
        Xu = torch.zeros(n * ld + 2, dtype=torch.float64, device="cuda")  # starts 8 bytes in
        Xu[1: 1 + n * ld].view(n, ld)[:, :nrhs] = dev(Xh)
        outs = []
        for X, ldx, ptr in ((Xa, ld, Xa.data_ptr()), (Xu, ld, Xu.data_ptr() + 8)):
            Y = torch.full((n * ld + 2,), np.nan, dtype=torch.float64, device="cuda")
            rc = lib.spx_spmm(A.handle, nrhs, ctypes.c_void_p(ptr), ldx, ctypes.c_void_p(Y.data_ptr()),
                              ld, None)
            assert rc == 0
            outs.append(host(Y[: n * ld].view(n, ld)[:, :nrhs]))
        assert np.array_equal(bits(outs[0]), bits(outs[1]))
        Yr = orc.spmm(ref, Xh)
        for c in range(nrhs):
            spmv_within(outs[0][:, c], Yr[:, c], orc.abs_spmv(ref, Xh[:, c]))


@pytest.mark.parametrize("n", [1, 5, 31, 33])
def test_spmm_fewer_rows_than_a_block(orc, n):
    """Matrices with fewer rows than one 32-row block of the staged kernel
    (and one just over): 16 contiguous columns against the oracle."""
    spx = require_gpu()
    rng = np.random.default_rng(70 + n)
    i = rng.integers(0, n, 6 * n).astype(np.int32)
    j = rng.integers(0, n, 6 * n).astype(np.int32)
    v = rng.uniform(-1, 1, i.size)
    prob = W.CooProblem(n=n, i=i, j=j, v=v)
    A = assemble(spx, prob)
    ref = orc.assemble(n, i, j, v)
    Xh = rng.uniform(-1, 1, (n, 16))
    Y = host(A.spmm(dev(Xh)))
    Yr = orc.spmm(ref, Xh)
    for c in range(16):
        spmv_within(Y[:, c], Yr[:, c], orc.abs_spmv(ref, Xh[:, c]))


@pytest.mark.parametrize("nrhs", [8, 13, 16, 32, 64, 65])
def test_spmm_staged_runs_and_fallback(orc, nrhs):
    """The staged-run kernel (8 or more columns, 16-byte aligned X and Y):
    blocks whose run of entries fits the LDS stage and blocks that read their
    pairs from global memory (32 rows of 60 entries overflow it), empty rows,
    a ragged last block, contiguous X (one pass) and padded leading
    dimensions, more than 64 columns (two column chunks, an odd last
    column).  Bitwise the one-column-per-lane kernel, within the SpMV
    tolerance of the oracle."""
    import ctypes
    spx = require_gpu()
    lib = spx.load_library()
    rng = np.random.default_rng(35 + nrhs)
    n = 3001
    lengths = np.where(np.arange(n) % 11 == 0, 0, np.where((np.arange(n) // 32) % 5 == 1, 60, 9))
    i = np.repeat(np.arange(n, dtype=np.int32), lengths)
    j = rng.integers(0, n, i.size).astype(np.int32)
    v = rng.uniform(-1, 1, i.size)
    prob = W.CooProblem(n=n, i=i, j=j, v=v)
    A = assemble(spx, prob)
    ref = orc.assemble(n, i, j, v)
    Xh = rng.uniform(-1, 1, (n, nrhs))
    Yr = orc.spmm(ref, Xh)
    outs = []
    for ld, shift in ((nrhs, 0), (nrhs + 2 if nrhs % 2 == 0 else nrhs + 1, 0), (nrhs + 1, 1)):
        Xa = torch.zeros(n * ld + 2, dtype=torch.float64, device="cuda")
        Xa[shift: shift + n * ld].view(n, ld)[:, :nrhs] = dev(Xh)
        Y = torch.full((n * ld + 2,), np.nan, dtype=torch.float64, device="cuda")
        rc = lib.spx_spmm(A.handle, nrhs, ctypes.c_void_p(Xa.data_ptr() + 8 * shift), ld,
                          ctypes.c_void_p(Y.data_ptr()), ld, None)
        assert rc == 0
        Yo = host(Y[: n * ld].view(n, ld))
        assert np.isnan(Yo[:, nrhs:]).all()  # padding untouched
        outs.append(Yo[:, :nrhs])
    for o in outs[1:]:
        assert np.array_equal(bits(o), bits(outs[0]))
    for c in range(nrhs):
        spmv_within(outs[0][:, c], Yr[:, c], orc.abs_spmv(ref, Xh[:, c]))


def _row_set_pattern(rng, tiles, tail):
    """Tiles of 32 rows of five kinds, in turn: 9 random columns a row (the
    tile's rows of X staged), 12 (too many distinct columns: gathered), rows
    of 0..65 entries from a 100-column window (staged, rows longer than one
    32-entry chunk), 40 a row (too many entries: gathered), and no entries;
    then a ragged last tile."""
    n = 32 * tiles + tail
    I, J = [], []
    cycle = [0, 1, 31, 32, 33, 64, 65, 16, 17, 2]
    for r in range(n):
        kind = (r // 32) % 5
        if kind == 0:
            cols = rng.choice(n, 9, replace=False)
        elif kind == 1:
            cols = rng.choice(n, 12, replace=False)
        elif kind == 2:
            lo = min(max(r - 50, 0), n - 100)
            cols = lo + rng.choice(100, cycle[r % len(cycle)], replace=False)
        elif kind == 3:
            cols = rng.choice(n, 40, replace=False)
        else:
            cols = np.zeros(0, np.int64)
        I.append(np.full(cols.size, r))
        J.append(cols)
    i = np.concatenate(I).astype(np.int32)
    j = np.concatenate(J).astype(np.int32)
    return W.CooProblem(n=n, i=i, j=j, v=rng.uniform(-1, 1, i.size))


def _spmm16(lib, A, Xh, ld):
    import ctypes
    n = Xh.shape[0]
    Xa = torch.zeros(n * ld + 2, dtype=torch.float64, device="cuda")
    Xa[: n * ld].view(n, ld)[:, :16] = dev(Xh)
    Y = torch.full((n * ld + 2,), np.nan, dtype=torch.float64, device="cuda")
    rc = lib.spx_spmm(A.handle, 16, ctypes.c_void_p(Xa.data_ptr()), ld,
                      ctypes.c_void_p(Y.data_ptr()), ld, None)
    assert rc == 0
    return host(Y[: n * ld].view(n, ld)[:, :16])


@pytest.mark.parametrize("tiles,tail", [(40, 7), (5, 0), (0, 9)])
def test_spmm16_row_set_tiles(orc, tiles, tail):
    """The 16-column product with each tile's rows of X staged in LDS (16
    contiguous columns): every kind of tile, bitwise equal to the paired-
    column kernel (16 columns at leading dimension 18) and within the SpMV
    tolerance of the oracle; a second product reuses the index."""
    spx = require_gpu()
    lib = spx.load_library()
    rng = np.random.default_rng(90 + tiles)
    prob = _row_set_pattern(rng, tiles, tail)
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    for rep in range(2):
        Xh = rng.uniform(-1, 1, (prob.n, 16))
        Ys = _spmm16(lib, A, Xh, 16)
        Yp = _spmm16(lib, A, Xh, 18)
        assert np.array_equal(bits(Ys), bits(Yp)), rep
        Yr = orc.spmm(ref, Xh)
        for c in range(16):
            spmv_within(Ys[:, c], Yr[:, c], orc.abs_spmv(ref, Xh[:, c]))


def test_spmm16_tile_heights_same_bits(orc):
    """16-, 32- and 64-row tiles (the index rebuilt at each change) give the
    same bits as the paired-column kernel; the autotuner leaves one of them
    set; other heights are refused."""
    spx = require_gpu()
    from paper_2406_08646_amd import autotune
    lib = spx.load_library()
    rng = np.random.default_rng(95)
    prob = _row_set_pattern(rng, 30, 11)
    A = assemble(spx, prob)
    Xh = rng.uniform(-1, 1, (prob.n, 16))
    Yp = _spmm16(lib, A, Xh, 18)
    assert A.get_option(spx.OPT_SPMM_TILE_ROWS) == 32
    for rows in (16, 64, 32, 16):
        A.set_option(spx.OPT_SPMM_TILE_ROWS, rows)
        assert A.get_option(spx.OPT_SPMM_TILE_ROWS) == rows
        assert np.array_equal(bits(_spmm16(lib, A, Xh, 16)), bits(Yp)), rows
    with pytest.raises(spx.SpxError) as e:
        A.set_option(spx.OPT_SPMM_TILE_ROWS, 48)
    assert e.value.code == spx.INVALID_ARG
    best = autotune.tune_spmm(A, dev(Xh), repeats=2)
    assert best["rows"] in (16, 32, 64) and A.get_option(spx.OPT_SPMM_TILE_ROWS) == best["rows"]
    assert np.array_equal(bits(_spmm16(lib, A, Xh, 16)), bits(Yp))


def test_spmm16_row_set_non_finite_x(orc):
    """Rows of X holding inf and NaN: only the rows of Y whose entries name
    them turn non-finite (a chunk's unused slots add +0.0 times a row of
    zeros, never a staged row), and the bits match the paired-column
    kernel's."""
    spx = require_gpu()
    lib = spx.load_library()
    rng = np.random.default_rng(97)
    prob = _row_set_pattern(rng, 12, 5)
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    Xh = rng.uniform(-1, 1, (prob.n, 16))
    k_inf, k_nan = int(prob.j[0]), int(prob.j[prob.j.size // 2])
    Xh[k_inf, :] = np.inf
    Xh[k_nan, 5] = np.nan
    Ys = _spmm16(lib, A, Xh, 16)
    Yp = _spmm16(lib, A, Xh, 18)
    fin = np.isfinite(Yp)
    assert np.array_equal(fin, np.isfinite(Ys))
    assert np.array_equal(np.isnan(Yp), np.isnan(Ys))
    assert np.array_equal(bits(Ys[fin]), bits(Yp[fin]))
    assert np.array_equal(Ys[np.isinf(Yp)], Yp[np.isinf(Yp)])
    touched = np.zeros(prob.n, bool)
    touched[prob.i[(prob.j == k_inf) | (prob.j == k_nan)]] = True
    assert np.isfinite(Ys[~touched]).all()
    Xf = Xh.copy()
    Xf[k_inf, :] = 0.0
    Xf[k_nan, 5] = 0.0
    Yr = orc.spmm(ref, Xf)
    for c in range(16):
        rows = ~touched
        spmv_within(Ys[rows, c], Yr[rows, c], orc.abs_spmv(ref, Xf[:, c])[rows])


def test_sddmm_and_gather_bitwise(orc):
    spx = require_gpu()
    rng = np.random.default_rng(32)
    prob = W.random_coo(rng, 3000, 60000, neg_frac=0.2, extreme=False)
    A = assemble(spx, prob)
    ref = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    lam, u = rng.uniform(-1, 1, (2, prob.n))
    G = A.sddmm(dev(lam), dev(u))
    assert np.array_equal(bits(host(G)), bits(orc.sddmm(ref, lam, u)))
    gv = A.coo_gather(G)
    assert np.array_equal(bits(host(gv)), bits(orc.coo_grad(prob.i, prob.j, lam, u)))


def test_gather_blocks_bitwise(orc):
    spx = require_gpu()
    prob, theta, _, _ = W.config5(N=32)
    A = assemble(spx, prob)
    rng = np.random.default_rng(33)
    lam, u = rng.uniform(-1, 1, (2, prob.n))
    G = A.sddmm(dev(lam), dev(u))
    ge = A.coo_gather_blocks(G, dev(prob.dv_dlogk), 16)
    gv = orc.coo_grad(prob.i, prob.j, lam, u)
    assert np.array_equal(bits(host(ge)), bits(orc.block_reduce(gv, prob.dv_dlogk, 16)))


def test_torch_allocator_hook():
    """With PyTorch's caching allocator installed, the library's memory shows
    up in torch's accounting, results are bitwise those of hipMalloc'd
    handles, and blocks go back to the allocator that made them even when the
    hook changes in between."""
    spx = require_gpu()
    prob, x, b = W.config1()
    A0 = assemble(spx, prob)
    y0 = host(A0.matmult(dev(x)))
    r0 = A0.cg_solve(dev(b), rtol=1e-10)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    spx.use_torch_allocator(True)
    try:
        A1 = assemble(spx, prob)
        y1 = host(A1.matmult(dev(x)))
        r1 = A1.cg_solve(dev(b), rtol=1e-10)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() > before + 36100 * 12
        assert np.array_equal(bits(y1), bits(y0))
        assert r1.iters == r0.iters and np.array_equal(bits(host(r1.x)), bits(host(r0.x)))
        batch = spx.batch_create([A1])
        xb, it, rel, st = batch.batch_cg(dev(b), rtol=1e-8)
        assert st == 0
    finally:
        spx.use_torch_allocator(False)
    # the hook-made blocks are freed through torch after the hook is gone
    batch.destroy()
    A1.destroy()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + 4 * 1024 * 1024
    A2 = assemble(spx, prob)
    assert np.array_equal(bits(host(A2.matmult(dev(x)))), bits(y0))


@pytest.mark.parametrize("n", [0, 1, 7, 4096, 1_000_003])
def test_bandwidth_reference_kernels(n):
    spx = require_gpu()
    x = np.random.default_rng(60 + n % 97).uniform(-1, 1, n)
    xd = dev(x)
    y = torch.full_like(xd, np.nan)
    spx.stream_copy(xd, y)
    assert np.array_equal(bits(host(y)), bits(x))
    parts = host(spx.stream_sum(xd))
    assert abs(parts.sum() - x.sum()) <= 1e-12 * max(1.0, np.abs(x).sum())
