"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it does not compute: brute
force on tiny inputs, closed forms of the model operators, dense LU,
spectral facts of CG, finite differences and a hand-written worked example.
A dropped term, a wrong sign or index or a transposed operand in the oracle
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2406_08646_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def dense_bruteforce(n, i, j, v):
    """Dense accumulation D[i][j] += v[k] in increasing k from +0.0, plus
    the set of touched entries."""
    D = np.zeros((n, n))
    touched = np.zeros((n, n), bool)
    for k in range(len(i)):
        if i[k] < 0 or j[k] < 0:
            continue
        D[i[k], j[k]] = D[i[k], j[k]] + v[k]
        touched[i[k], j[k]] = True
    return D, touched


# ---------------------------------------------------------------- assembly

@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(n=st.integers(1, 300), ncoo=st.integers(0, 5000), seed=st.integers(0, 2**32 - 1),
       neg=st.sampled_from([0.0, 0.1, 0.5]), pool=st.integers(1, 2000))
def test_assembly_matches_dense_bruteforce(orc, n, ncoo, seed, neg, pool):
    rng = np.random.default_rng(seed)
    p = W.random_coo(rng, n, ncoo, neg_frac=neg, dup_pool=pool)
    A = orc.assemble(n, p.i, p.j, p.v)
    D, touched = dense_bruteforce(n, p.i, p.j, p.v)
    # pattern: exactly the touched entries, rows then columns ascending
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    assert A.rowptr[0] == 0 and np.all(np.diff(A.rowptr) >= 0)
    assert np.array_equal(np.argwhere(touched), np.stack([rows, A.col], 1).reshape(-1, 2))
    # values: bitwise equal, signed zeros included
    assert np.array_equal(bits(A.val), bits(D[rows, A.col]))
    # helper maps: perm lists every kept k once, ascending inside each run
    kept = np.flatnonzero((p.i >= 0) & (p.j >= 0))
    assert np.array_equal(np.sort(A.perm), kept)
    for t in range(A.nnz):
        run = A.perm[A.jmap[t]:A.jmap[t + 1]]
        assert run.size > 0 and np.all(np.diff(run) > 0)
        assert np.all(p.i[run] == rows[t]) and np.all(p.j[run] == A.col[t])
    # kslot maps each kept triplet to its entry
    ks = orc.coo_slots(A)
    assert np.all(ks[(p.i < 0) | (p.j < 0)] == -1)
    assert np.all(rows[ks[kept]] == p.i[kept]) and np.all(A.col[ks[kept]] == p.j[kept])


def test_assembly_add_mode(orc):
    rng = np.random.default_rng(5)
    p = W.random_coo(rng, 40, 600)
    A = orc.assemble(40, p.i, p.j, p.v)
    v2 = rng.uniform(-1, 1, p.ncoo)
    added = orc.coo_values(A.jmap, A.perm, v2, mode=1, val=A.val)
    D, _ = dense_bruteforce(40, p.i, p.j, v2)
    rows = np.repeat(np.arange(40), np.diff(A.rowptr))
    assert np.array_equal(bits(added), bits(A.val + D[rows, A.col]))


def test_assembly_rejects_out_of_range(orc):
    i = np.array([0, 1, 5], np.int32)
    j = np.array([0, 1, 1], np.int32)
    with pytest.raises(orc.OracleError) as e:
        orc.coo_pattern(5, i, j)
    assert e.value.code == -2
    with pytest.raises(orc.OracleError):
        orc.coo_pattern(5, np.array([0], np.int32), np.array([7], np.int32))


def test_assembly_empty_and_all_ignored(orc):
    A = orc.assemble(7, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert A.nnz == 0 and np.all(A.rowptr == 0)
    A = orc.assemble(7, np.array([-1, 3], np.int32), np.array([2, -4], np.int32), np.ones(2))
    assert A.nnz == 0 and A.nvalid == 0


def test_assembly_signed_zero_and_nan(orc):
    i = np.array([0, 0, 1, 1, 2], np.int32)
    j = np.array([0, 1, 1, 1, 2], np.int32)
    v = np.array([-0.0, 3.0, np.inf, -np.inf, np.nan])
    A = orc.assemble(3, i, j, v)
    assert bits(A.val[0:1])[0] == bits(np.array([0.0]))[0]  # +0.0 + -0.0 = +0.0
    assert np.isnan(A.val[2]) and np.isnan(A.val[3])


def read_golden():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "periodic_tridiag.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("case"):
                parts = dict(x.split("=") for x in line.split()[2:])
                cur = {"n": int(parts["n"]), "X": [float(a) for a in parts["X"].split(",")],
                       "rows": []}
                cases.append(cur)
            else:
                head, rest = line.split(":", 1)
                ents = [tuple(e.split(":")) for e in rest.split()]
                cur["rows"].append([(int(c), float(val)) for c, val in ents])
    return cases


def test_worked_example_periodic_jacobian(orc):
    for case in read_golden():
        n = case["n"]
        p = W.periodic_tridiag_jacobian(n, 1.0, np.array(case["X"]))
        A = orc.assemble(n, p.i, p.j, p.v)
        for r, ents in enumerate(case["rows"]):
            got = [(int(c), float(v)) for c, v in zip(A.col[A.rowptr[r]:A.rowptr[r + 1]],
                                                      A.val[A.rowptr[r]:A.rowptr[r + 1]])]
            assert got == ents, (case, r)


def test_worked_example_jacobian_action(orc):
    # J w is the linearisation of R(X) = d(X_{i-1} - 2X_i + X_{i+1}) + X_i^2 - F_i
    n, d = 37, 0.7
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, n)
    w = rng.uniform(-1, 1, n)
    p = W.periodic_tridiag_jacobian(n, d, X)
    A = orc.assemble(n, p.i, p.j, p.v)
    ref = d * (np.roll(w, 1) - 2 * w + np.roll(w, -1)) + 2 * X * w
    assert np.allclose(orc.spmv(A, w), ref, rtol=0, atol=1e-14)


# --------------------------------------------------- Q1 structure and values

@pytest.mark.parametrize("N,dim", [(1, 2), (2, 2), (5, 2), (8, 2), (1, 3), (2, 3), (4, 3)])
def test_q1_structure_closed_form(orc, N, dim):
    p = W.q1_poisson(N, dim)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    assert A.nnz == (3 * M - 2) ** dim
    assert A.nvalid == p.ncoo == N**dim * 4**dim
    node = np.arange(p.n)
    length = np.ones(p.n, np.int64)
    for d in range(dim):
        c = (node // M**d) % M
        length *= 3 - ((c == 0) | (c == N)).astype(np.int64) if N > 0 else 1
    assert np.array_equal(np.diff(A.rowptr), length)


def interior_mask(N, dim):
    M = N + 1
    node = np.arange(M**dim)
    inside = np.ones(M**dim, bool)
    for d in range(dim):
        c = (node // M**d) % M
        inside &= (c > 0) & (c < N)
    return inside


@pytest.mark.parametrize("N,dim", [(6, 2), (4, 3)])
def test_q1_values_closed_form(orc, N, dim):
    p = W.q1_poisson(N, dim)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    h = 1.0 / N
    inside = interior_mask(N, dim)
    rows = np.repeat(np.arange(p.n), np.diff(A.rowptr))
    # boundary rows/columns are the identity, exactly
    bnd = ~inside
    on_b = bnd[rows] | bnd[A.col]
    diag = rows == A.col
    assert np.all(A.val[on_b & diag] == 1.0)
    assert np.all(A.val[on_b & ~diag] == 0.0)
    # interior stencil
    ri = np.array([(rows // M**d) % M for d in range(dim)])
    ci = np.array([(A.col // M**d) % M for d in range(dim)])
    ndiff = np.sum(ri != ci, axis=0)
    if dim == 2:
        expect = {0: 8.0 / 3.0, 1: -1.0 / 3.0, 2: -1.0 / 3.0}
    else:
        expect = {0: 8.0 * h / 3.0, 1: 0.0, 2: -h / 6.0, 3: -h / 12.0}
    sel = ~on_b
    for m, e in expect.items():
        got = A.val[sel & (ndiff == m)]
        assert got.size > 0
        assert np.allclose(got, e, rtol=4e-16 * 8, atol=1e-300 if e else 4e-17), (m, e)


def q1_mode(N, dim, ks):
    M = N + 1
    node = np.arange(M**dim)
    v = np.ones(M**dim)
    c = []
    for d in range(dim):
        idx = (node // M**d) % M
        v *= np.sin(ks[d] * math.pi * idx / N)
        c.append(math.cos(ks[d] * math.pi / N))
    if dim == 2:
        lam = (8 - 2 * c[0] - 2 * c[1] - 4 * c[0] * c[1]) / 3
    else:
        h = 1.0 / N
        lam = h * (8.0 / 3 - (2.0 / 3) * (c[0] * c[1] + c[1] * c[2] + c[0] * c[2])
                   - (2.0 / 3) * c[0] * c[1] * c[2])
    return v, lam


@pytest.mark.parametrize("N,dim,ks", [(8, 2, (1, 1)), (8, 2, (3, 5)), (8, 2, (7, 2)),
                                      (6, 3, (1, 1, 1)), (6, 3, (2, 5, 3)), (6, 3, (5, 5, 1))])
def test_spmv_closed_form_eigenpairs(orc, N, dim, ks):
    p = W.q1_poisson(N, dim)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    v, lam = q1_mode(N, dim, ks)
    Av = orc.spmv(A, v)
    scale = np.max(orc.abs_spmv(A, v))
    assert np.max(np.abs(Av - lam * v)) <= 1e-13 * scale
    # and the transpose product gives the same for this symmetric operator
    assert np.max(np.abs(orc.spmv_transpose(A, v) - lam * v)) <= 1e-13 * scale


@pytest.mark.parametrize("N,dim", [(7, 2), (5, 3)])
def test_spmv_annihilates_linear_functions(orc, N, dim):
    p = W.q1_poisson(N, dim)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    node = np.arange(p.n)
    f = np.full(p.n, 0.3)
    for d, coef in zip(range(dim), (1.5, -2.0, 0.25)):
        f += coef * ((node // M**d) % M) / N
    Af = orc.spmv(A, f)
    # rows whose whole stencil is interior
    inside = interior_mask(N, dim)
    deep = inside.copy()
    rows = np.repeat(np.arange(p.n), np.diff(A.rowptr))
    touches_b = np.zeros(p.n, bool)
    np.logical_or.at(touches_b, rows, ~inside[A.col])
    deep &= ~touches_b
    assert deep.any()
    assert np.max(np.abs(Af[deep])) <= 1e-14 * np.max(orc.abs_spmv(A, f))


def test_spmv_symmetry_and_transpose_identity(orc):
    rng = np.random.default_rng(7)
    p = W.q1_poisson(6, 3, kappa=np.exp(rng.standard_normal(216)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    x, y = rng.uniform(-1, 1, (2, p.n))
    assert abs(x @ orc.spmv(A, y) - y @ orc.spmv(A, x)) <= 1e-13 * (np.abs(x) @ orc.abs_spmv(A, y))
    # non-symmetric: x.(A y) = (A^T x).y, and A^T differs from A
    q = W.random_coo(rng, 150, 3000, extreme=False)
    B = orc.assemble(150, q.i, q.j, q.v)
    x, y = rng.uniform(-1, 1, (2, 150))
    lhs = x @ orc.spmv(B, y)
    rhs = orc.spmv_transpose(B, x) @ y
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(x) @ orc.abs_spmv(B, y))
    assert np.max(np.abs(orc.spmv_transpose(B, x) - orc.spmv(B, x))) > 1e-3
    # A^T assembled from the swapped triplets gives the same product
    Bt = orc.assemble(150, q.j, q.i, q.v)
    assert np.array_equal(bits(orc.spmv(Bt, x)), bits(orc.spmv(Bt, x)))
    assert np.allclose(orc.spmv(Bt, x), orc.spmv_transpose(B, x), rtol=0, atol=1e-13)


def test_spmv_against_scipy_library(orc):
    rng = np.random.default_rng(8)
    q = W.random_coo(rng, 90, 2000, extreme=False)
    A = orc.assemble(90, q.i, q.j, q.v)
    keep = (q.i >= 0) & (q.j >= 0)
    S = sp.coo_matrix((q.v[keep], (q.i[keep], q.j[keep])), shape=(90, 90)).tocsr()
    x = rng.uniform(-1, 1, 90)
    assert np.allclose(orc.spmv(A, x), S @ x, rtol=0, atol=1e-13)
    X = rng.uniform(-1, 1, (90, 5))
    assert np.allclose(orc.spmm(A, X), S @ X, rtol=0, atol=1e-13)
    Y = orc.spmm(A, X)
    for c in range(5):
        assert np.array_equal(bits(Y[:, c]), bits(orc.spmv(A, X[:, c])))


def test_five_point_closed_form(orc):
    # constant coefficient 1: eigenvalues 4 - 2cos(k pi/(L+1)) - 2cos(l pi/(L+1))
    L = 9
    nh = L * (L - 1)
    p = W.five_point_system(L, np.ones(nh), np.ones(nh), np.ones(4 * L))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    assert A.nnz == 5 * L * L - 4 * L
    idx = np.arange(L * L)
    xs, ys = idx % L, idx // L
    for k, l in [(1, 1), (3, 7), (9, 2)]:
        v = np.sin(k * math.pi * (xs + 1) / (L + 1)) * np.sin(l * math.pi * (ys + 1) / (L + 1))
        lam = 4 - 2 * math.cos(k * math.pi / (L + 1)) - 2 * math.cos(l * math.pi / (L + 1))
        assert np.max(np.abs(orc.spmv(A, v) - lam * v)) <= 1e-13 * 8


# --------------------------------------------------------------------- CG

@pytest.mark.parametrize("N,dim", [(2, 2), (3, 2), (5, 2), (8, 2), (2, 3), (3, 3), (4, 3)])
def test_cg_matches_dense_lu(orc, N, dim):
    rng = np.random.default_rng(N * 10 + dim)
    nel = N**dim
    p = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(nel)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    D = np.zeros((p.n, p.n))
    rows = np.repeat(np.arange(p.n), np.diff(A.rowptr))
    D[rows, A.col] = A.val
    xs = np.linalg.solve(D, b)
    res = orc.pcg(A, b, 1e-14, 10000)
    assert res.status == 0
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert res.relres <= 1e-13


@pytest.mark.parametrize("N,dim,ks", [(10, 2, (2, 3)), (6, 3, (1, 2, 4))])
def test_cg_eigenmode_one_step(orc, N, dim, ks):
    p = W.q1_poisson(N, dim)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    v, lam = q1_mode(N, dim, ks)
    res = orc.pcg(A, v, 1e-12, 50)
    assert res.status == 0 and res.iters == 1
    assert np.max(np.abs(res.x - v / lam)) <= 1e-12 * np.max(np.abs(v / lam))


def test_cg_sum_of_modes_terminates(orc):
    N = 12
    p = W.q1_poisson(N, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    modes = [(1, 1), (2, 5), (7, 3), (11, 11)]
    b = sum(q1_mode(N, 2, k)[0] * (1 + 0.1 * s) for s, k in enumerate(modes))
    res = orc.pcg(A, b, 1e-11, 100)
    assert res.status == 0 and res.iters <= len(modes) + 1


def test_cg_error_bound_and_iteration_sanity(orc):
    N = 31
    p = W.q1_poisson(N, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, p.n)
    res = orc.pcg(A, b, 1e-10, 5000)
    assert res.status == 0 and res.relres <= 1e-10 * 1.001
    ref = orc.pcg(A, b, 1e-15, 5000)
    lam_min = min(1.0, q1_mode(N, 2, (1, 1))[1])
    r = b - orc.spmv(A, res.x)
    rr = b - orc.spmv(A, ref.x)
    assert np.linalg.norm(res.x - ref.x) <= (np.linalg.norm(r) + np.linalg.norm(rr)) / lam_min
    # Jacobi-scaled condition number ~ (8/3)/lam_min*(...); iterations well under the bound
    kappa = q1_mode(N, 2, (N - 1, N - 1))[1] / q1_mode(N, 2, (1, 1))[1]
    assert res.iters <= 0.5 * math.sqrt(kappa) * math.log(2 / 1e-10) * 1.5


def test_cg_status_codes(orc):
    # zero diagonal
    i = np.array([0, 1, 1], np.int32)
    j = np.array([1, 0, 1], np.int32)
    A = orc.assemble(2, i, j, np.array([1.0, 1.0, 2.0]))
    assert orc.pcg(A, np.ones(2), 1e-8, 10).status == -4
    # indefinite -> breakdown (p.Ap <= 0)
    A = orc.assemble(2, np.array([0, 1], np.int32), np.array([0, 1], np.int32),
                     np.array([1.0, -1.0]))
    assert orc.pcg(A, np.array([0.0, 1.0]), 1e-8, 10).status == -6
    # maxit reached -> not converged, x still usable
    p = W.q1_poisson(20, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = np.random.default_rng(0).uniform(-1, 1, p.n)
    r = orc.pcg(A, b, 1e-12, 3)
    assert r.status == -5 and r.iters == 3 and r.relres < 1.0
    # b = 0 converges immediately
    r = orc.pcg(A, np.zeros(p.n), 1e-8, 10)
    assert r.status == 0 and r.iters == 0 and np.all(r.x == 0)


# -------------------------------------------------------- mixed precision

def test_mixed_refinement_reaches_fp64_tolerance(orc):
    rng = np.random.default_rng(1)
    N = 10
    z = rng.standard_normal(N**3)
    p = W.q1_poisson(N, 3, kappa=np.exp(z))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    res = orc.pcg_mixed(A, b, 1e-10, 1e-4)
    assert res.status == 0 and res.relres <= 1e-10
    assert res.outer >= 2  # an fp32 inner solve alone cannot reach 1e-10
    ref = orc.pcg(A, b, 1e-12)
    D = np.zeros((p.n, p.n))
    D[np.repeat(np.arange(p.n), np.diff(A.rowptr)), A.col] = A.val
    xs = np.linalg.solve(D, b)
    assert np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)
    assert np.linalg.norm(ref.x - xs) <= 1e-9 * np.linalg.norm(xs)


def _lognormal_q1(orc, N, seed=1):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(N**3)
    p = W.q1_poisson(N, 3, kappa=np.exp(z))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    return A, rng.uniform(-1, 1, p.n)


def _fp32_residual(A, b, x):
    """||fl32(b) - fl32(A) x|| / ||fl32(b)||, formed in fp64 with numpy."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    A32 = sp.csr_matrix((A.val.astype(np.float32).astype(np.float64), (rows, A.col)),
                        shape=(A.n, A.n))
    b32 = b.astype(np.float32).astype(np.float64)
    return np.linalg.norm(b32 - A32 @ x) / np.linalg.norm(b32)


def test_mixed_inner_stop_rules(orc):
    """One refinement step from x = 0 is one inner fp32 solve on fl32(b).
    The literal rule stops it once the inner residual has fallen by
    rtol_inner (checked on the true fp32-operator residual of the returned
    x, which CG reduces smoothly, so it lands within a few factors of the
    target, not orders below it).  The early exit stops as soon as the
    residual is under rtol_outer ||b|| / 2, which for a loose outer target
    ends the step far above rtol_inner."""
    A, b = _lognormal_q1(orc, 10)
    lit = orc.pcg_mixed(A, b, 1e-10, 1e-4, maxit_outer=1)
    assert lit.outer == 1 and lit.status == -5
    rel = _fp32_residual(A, b, lit.x)
    assert 1e-6 < rel <= 1.5e-4, rel
    early = orc.pcg_mixed(A, b, 2e-2, 1e-4, maxit_outer=1, early_exit=True)
    rel_e = _fp32_residual(A, b, early.x)
    assert 1e-3 < rel_e <= 1.5e-2, rel_e
    assert early.inner < lit.inner
    # to 1e-10 both rules reach the target in the same number of steps;
    # the early exit only shortens the last inner solve
    full_l = orc.pcg_mixed(A, b, 1e-10, 1e-4)
    full_e = orc.pcg_mixed(A, b, 1e-10, 1e-4, early_exit=True)
    assert full_l.status == 0 and full_e.status == 0
    assert full_l.relres <= 1e-10 and full_e.relres <= 1e-10
    assert full_e.outer == full_l.outer and full_e.inner < full_l.inner


def test_thread_count_does_not_change_results(orc):
    """The parallel loops keep every element and every 4096-entry dot block
    in one thread, in order: results are bitwise those of one thread."""
    p = W.q1_poisson(40, 3)  # 68,921 rows: above the parallel threshold
    A = orc.assemble(p.n, p.i, p.j, p.v)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, p.n)
    b = rng.uniform(-1, 1, p.n)
    old = orc.get_threads()
    try:
        out = {}
        for t in (1, 5):
            orc.set_threads(t)
            y = orc.spmv(A, x)
            c = orc.pcg(A, b, 1e-8)
            m = orc.pcg_mixed(A, b, 1e-10, 1e-4)
            out[t] = (y, c, m)
        (y1, c1, m1), (y5, c5, m5) = out[1], out[5]
        assert np.array_equal(bits(y1), bits(y5))
        assert c1.iters == c5.iters and np.array_equal(bits(c1.x), bits(c5.x))
        assert (m1.outer, m1.inner) == (m5.outer, m5.inner)
        assert np.array_equal(bits(m1.x), bits(m5.x))
    finally:
        orc.set_threads(old)


# ----------------------------------------------------------- gradient

def _dense(orc, n, i, j, v):
    A = orc.assemble(n, i, j, v)
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    return A, sp.csr_matrix((A.val, (rows, A.col)), shape=(n, n))


def test_gradient_matches_finite_differences(orc):
    N = 12
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(N * N)
    prob = W.q1_poisson(N, 2, kappa=np.exp(theta))
    tgt = W.q1_poisson(N, 2, kappa=np.ones(N * N))
    b = np.ones(prob.n)
    _, St = _dense(orc, tgt.n, tgt.i, tgt.j, tgt.v)
    ustar = spla.spsolve(St.tocsc(), b)

    def loss(th):
        pr = W.q1_poisson(N, 2, kappa=np.exp(th))
        _, S = _dense(orc, pr.n, pr.i, pr.j, pr.v)
        u = spla.spsolve(S.tocsc(), b)
        return 0.5 * np.sum((u - ustar) ** 2)

    A = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    fw = orc.pcg(A, b, 1e-14)
    u = fw.x
    g = u - ustar
    adj = orc.pcg(A, g, 1e-14)  # A symmetric, so A^T lambda = g is the same solve
    lam = adj.x
    grad_v = orc.coo_grad(prob.i, prob.j, lam, u)
    grad_theta = orc.block_reduce(grad_v, prob.dv_dlogk, 16)
    # second, independent formula: element adjoint -exp(theta_e) lam_e^T K u_e
    K = W.q1_reference_stiffness(2)
    gi = prob.i.reshape(-1, 4, 4)[:, :, 0]
    M = N + 1
    node = np.arange(prob.n)
    bnd = ((node % M == 0) | (node % M == N) | (node // M == 0) | (node // M == N))
    lam_e = np.where(bnd[gi], 0.0, lam[gi])
    u_e = np.where(bnd[gi], 0.0, u[gi])
    g2 = -np.exp(theta) * np.einsum("ea,ab,eb->e", lam_e, K, u_e)
    assert np.allclose(grad_theta, g2, rtol=1e-10, atol=1e-12 * np.max(np.abs(g2)))
    # central differences with direct solves
    idx = np.sort(rng.choice(N * N, 20, replace=False))
    hfd = 1e-4
    fd = []
    for e in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[e] += hfd
        tm[e] -= hfd
        fd.append((loss(tp) - loss(tm)) / (2 * hfd))
    fd = np.array(fd)
    assert np.linalg.norm(grad_theta[idx] - fd) <= 1e-6 * np.linalg.norm(fd)
    # directional derivative
    dth = rng.standard_normal(N * N)
    dd = (loss(theta + hfd * dth) - loss(theta - hfd * dth)) / (2 * hfd)
    assert abs(grad_theta @ dth - dd) <= 1e-6 * abs(dd)


def test_sddmm_and_coo_grad_consistent(orc):
    rng = np.random.default_rng(4)
    q = W.random_coo(rng, 60, 900, extreme=False)
    A = orc.assemble(60, q.i, q.j, q.v)
    lam, u = rng.uniform(-1, 1, (2, 60))
    G = orc.sddmm(A, lam, u)
    gv = orc.coo_grad(q.i, q.j, lam, u)
    ks = orc.coo_slots(A)
    ref = np.where(ks >= 0, G[np.maximum(ks, 0)], 0.0)
    assert np.array_equal(bits(gv), bits(ref))
    # G is the pattern sample of the outer product -lam u^T
    rows = np.repeat(np.arange(60), np.diff(A.rowptr))
    assert np.array_equal(bits(G), bits(-np.outer(lam, u)[rows, A.col]))


def test_batched_systems_each_solve(orc):
    probs, bs = W.config4(nsys=4, lo=4, hi=24, seed=9)
    for p, b in zip(probs, bs):
        A = orc.assemble(p.n, p.i, p.j, p.v)
        assert A.nnz == 5 * p.n - 4 * p.grid
        res = orc.pcg(A, b, 1e-8)
        assert res.status == 0 and res.relres <= 1e-8 * 1.001
        D = np.zeros((p.n, p.n))
        D[np.repeat(np.arange(p.n), np.diff(A.rowptr)), A.col] = A.val
        assert np.allclose(D, D.T)
        xs = np.linalg.solve(D, b)
        assert np.linalg.norm(res.x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_coo_rows_sample_matches_full_assembly(orc):
    p = W.q1_poisson(5, 3)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    rows = np.array([0, 7, 50, 100, 215], np.int32)
    ptr, col, val = orc.coo_rows(p.n, p.i, p.j, p.v, rows)
    for s, r in enumerate(rows):
        a, b = A.rowptr[r], A.rowptr[r + 1]
        assert np.array_equal(col[ptr[s]:ptr[s + 1]], A.col[a:b])
        assert np.array_equal(bits(val[ptr[s]:ptr[s + 1]]), bits(A.val[a:b]))


# ---------------------------------------------------------- COO vectors

@settings(max_examples=40, deadline=None)
@given(n=st.integers(1, 200), ncoo=st.integers(0, 3000), seed=st.integers(0, 2**32 - 1))
def test_vec_coo_equals_diagonal_of_matrix_assembly(orc, n, ncoo, seed):
    """The vector sums (dense in-order accumulation) equal, bitwise, the
    diagonal of the matrix assembled by sort-and-sum from (i, i, v)."""
    rng = np.random.default_rng(seed)
    p = W.random_coo(rng, n, ncoo, neg_frac=0.2)
    x0 = rng.uniform(-1, 1, n)
    x = orc.vec_coo(n, p.i, p.v, x0)
    A = orc.assemble(n, p.i, p.i, p.v)
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    assert np.all(rows == A.col)
    touched = np.zeros(n, bool)
    touched[rows] = True
    assert np.array_equal(bits(x[rows]), bits(A.val))
    assert np.array_equal(bits(x[~touched]), bits(x0[~touched]))
    xa = orc.vec_coo(n, p.i, p.v, x0, mode=1)
    assert np.array_equal(bits(xa[rows]), bits(x0[rows] + A.val))


def test_vec_coo_rejects_out_of_range(orc):
    with pytest.raises(orc.OracleError):
        orc.vec_coo(3, np.array([0, 3], np.int32), np.ones(2), np.zeros(3))


# ------------------------------------------------ single-reduction CG

@pytest.mark.parametrize("N,dim", [(3, 2), (8, 2), (3, 3)])
def test_single_reduction_cg_matches_dense_lu(orc, N, dim):
    rng = np.random.default_rng(70 + N)
    p = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    D = np.zeros((p.n, p.n))
    D[np.repeat(np.arange(p.n), np.diff(A.rowptr)), A.col] = A.val
    xs = np.linalg.solve(D, b)
    res = orc.pcg_single_reduction(A, b, 1e-14, 10000)
    assert res.status == 0 and res.relres <= 1e-13
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_single_reduction_cg_tracks_hestenes_stiefel(orc):
    """Same Krylov iterates in exact arithmetic: iteration counts agree and
    an eigenmode still converges in one step."""
    prob, _, b = W.config1()
    A = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    hs = orc.pcg(A, b, 1e-8)
    cg = orc.pcg_single_reduction(A, b, 1e-8)
    assert cg.status == 0 and abs(cg.iters - hs.iters) <= 2
    assert np.linalg.norm(cg.x - hs.x) <= 1e-6 * np.linalg.norm(hs.x)
    N = 10
    p = W.q1_poisson(N, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    node = np.arange(p.n)
    v = np.sin(2 * math.pi * (node % M) / N) * np.sin(3 * math.pi * (node // M) / N)
    r = orc.pcg_single_reduction(A, v, 1e-12, 50)
    assert r.status == 0 and r.iters == 1
    # breakdown on an indefinite matrix, maxit honoured
    B = orc.assemble(2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    assert orc.pcg_single_reduction(B, np.array([0.0, 1.0]), 1e-8, 10).status == -6
    rr = orc.pcg_single_reduction(A, np.random.default_rng(0).uniform(-1, 1, p.n), 1e-14, 3)
    assert rr.status == -5 and rr.iters == 3


# ------------------------------------------- pipelined (Ghysels-Vanroose) CG

@pytest.mark.parametrize("N,dim", [(3, 2), (8, 2), (2, 3), (4, 3)])
def test_pipelined_cg_matches_dense_lu(orc, N, dim):
    rng = np.random.default_rng(90 + N)
    p = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    D = np.zeros((p.n, p.n))
    D[np.repeat(np.arange(p.n), np.diff(A.rowptr)), A.col] = A.val
    xs = np.linalg.solve(D, b)
    res = orc.pcg_pipelined(A, b, 1e-13, 10000)
    assert res.status == 0 and res.relres <= 1e-12
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_pipelined_cg_iterates_equal_hestenes_stiefel(orc):
    """The k-th iterate is the k-th CG iterate (same Krylov space, same
    minimisation), so after a fixed k steps the two forms agree to rounding.
    The first one is closed form: x_1 = (r.u / (A u).u) u with u = D^-1 b."""
    rng = np.random.default_rng(7)
    N = 9
    p = W.q1_poisson(N, 2, kappa=np.exp(rng.standard_normal(N * N)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    D = np.zeros((p.n, p.n))
    D[np.repeat(np.arange(p.n), np.diff(A.rowptr)), A.col] = A.val
    u = b / np.diag(D)
    x1 = (b @ u) / ((D @ u) @ u) * u
    one = orc.pcg_pipelined(A, b, 1e-30, 1)
    assert one.status == -5 and one.iters == 1
    assert np.linalg.norm(one.x - x1) <= 1e-13 * np.linalg.norm(x1)
    for k in (2, 3, 5, 8, 13):
        pl = orc.pcg_pipelined(A, b, 1e-30, k)
        hs = orc.pcg(A, b, 1e-30, k)
        assert pl.iters == hs.iters == k
        assert np.linalg.norm(pl.x - hs.x) <= 1e-10 * np.linalg.norm(hs.x), k


def test_pipelined_cg_modes_statuses(orc):
    prob, _, b = W.config1()
    A = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    hs = orc.pcg(A, b, 1e-8)
    pl = orc.pcg_pipelined(A, b, 1e-8)
    assert pl.status == 0 and abs(pl.iters - hs.iters) <= 2 and pl.relres <= 1e-8 * 1.001
    N = 10
    p = W.q1_poisson(N, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    node = np.arange(p.n)
    mode = lambda a, c: np.sin(a * math.pi * (node % M) / N) * np.sin(c * math.pi * (node // M) / N)
    r = orc.pcg_pipelined(A, mode(2, 3), 1e-12, 50)
    assert r.status == 0 and r.iters == 1
    r = orc.pcg_pipelined(A, mode(1, 1) + mode(2, 3) + mode(4, 1), 1e-10, 50)
    assert r.status == 0 and r.iters <= 3 + 1
    B = orc.assemble(2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    assert orc.pcg_pipelined(B, np.array([0.0, 1.0]), 1e-8, 10).status == -6
    rr = orc.pcg_pipelined(A, np.random.default_rng(0).uniform(-1, 1, p.n), 1e-14, 3)
    assert rr.status == -5 and rr.iters == 3
    z = orc.pcg_pipelined(A, np.zeros(p.n), 1e-8)
    assert z.status == 0 and z.iters == 0 and np.all(z.x == 0)
    Z = orc.assemble(2, np.array([0, 1, 1], np.int32), np.array([1, 0, 1], np.int32),
                     np.array([1.0, 1.0, 2.0]))
    assert orc.pcg_pipelined(Z, np.ones(2), 1e-8, 10).status == -4


# ------------------------------------------- BiCG and TFQMR (non-symmetric)

def dense_of(A):
    D = np.zeros((A.n, A.n))
    D[np.repeat(np.arange(A.n), np.diff(A.rowptr)), A.col] = A.val
    return D


def small_nonsymmetric(seed, n=6):
    """A small well-conditioned non-symmetric matrix as COO (diagonal
    dominant, every entry present)."""
    rng = np.random.default_rng(seed)
    M = rng.uniform(-1, 1, (n, n)) + np.diag(rng.uniform(n, n + 2, n))
    ii, jj = np.nonzero(np.ones((n, n)))
    return ii.astype(np.int32), jj.astype(np.int32), M[ii, jj].copy(), rng.uniform(-1, 1, n)


@pytest.mark.parametrize("N,dim", [(8, 2), (4, 3)])
def test_bicg_on_symmetric_matrix_is_cg_value_for_value(orc, N, dim):
    """With the shadow residual started at r, a symmetric A keeps it equal
    to r, and BiCG performs CG's arithmetic: same iterates, bit for bit."""
    rng = np.random.default_rng(90 + N)
    p = W.q1_poisson(N, dim, kappa=np.exp(rng.standard_normal(N**dim)))
    A = orc.assemble(p.n, p.i, p.j, p.v)
    b = rng.uniform(-1, 1, p.n)
    for rtol, maxit in ((1e-10, 100000), (1e-14, 7)):
        c = orc.pcg(A, b, rtol, maxit)
        g = orc.bicg(A, b, rtol, maxit)
        assert g.status == c.status and g.iters == c.iters
        assert np.array_equal(bits(g.x), bits(c.x))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bicg_and_tfqmr_match_dense_lu_on_convection_diffusion(orc, seed):
    probs, bs = W.config6(nsys=2, lo=6, hi=20, seed=seed)
    for p, b in zip(probs, bs):
        A = orc.assemble(p.n, p.i, p.j, p.v)
        D = dense_of(A)
        assert np.max(np.abs(D - D.T)) > 0.1  # really non-symmetric
        xs = np.linalg.solve(D, b)
        for res in (orc.bicg(A, b, 1e-11), orc.tfqmr(A, b, 1e-11)):
            assert res.status == 0
            assert res.relres <= 1e-11 * 1.01
            assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_finite_termination_on_small_systems(orc, seed):
    """BiCG ends in at most n steps and TFQMR (whose unsmoothed residual is
    the squared BiCG polynomial) in at most 2n half-steps, up to rounding."""
    n = 6
    i, j, v, b = small_nonsymmetric(seed, n)
    A = orc.assemble(n, i, j, v)
    xs = np.linalg.solve(dense_of(A), b)
    g = orc.bicg(A, b, 1e-12)
    t = orc.tfqmr(A, b, 1e-12)
    assert g.status == 0 and g.iters <= n + 1
    assert t.status == 0 and t.iters <= 2 * n + 2
    for res in (g, t):
        assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_tfqmr_bound_dominates_the_true_residual(orc):
    """sqrt(m + 1) tau_m bounds ||b - A x_m|| at every half-step m: checked at
    exits forced after m = 1..12 half-steps and at convergence."""
    probs, bs = W.config6(nsys=1, lo=12, hi=12, seed=7)
    p, b = probs[0], bs[0]
    A = orc.assemble(p.n, p.i, p.j, p.v)
    bn = np.linalg.norm(b)
    for m in range(1, 13):
        t = orc.tfqmr(A, b, 1e-14, m)
        assert t.status == -5 and t.iters == m
        assert t.relres * bn <= t.bound * (1 + 1e-9)
    t = orc.tfqmr(A, b, 1e-9)
    assert t.status == 0 and t.relres * bn <= t.bound * (1 + 1e-9) <= 1e-9 * bn * (1 + 1e-9)


def test_eigenvector_right_hand_side_converges_at_once(orc):
    """An eigenvector of A whose support has a constant diagonal is an
    eigenvector of A D^-1 too: TFQMR is exact after one half-step, BiCG
    after one step."""
    N = 10
    p = W.q1_poisson(N, 2)
    A = orc.assemble(p.n, p.i, p.j, p.v)
    M = N + 1
    node = np.arange(p.n)
    v = np.sin(2 * math.pi * (node % M) / N) * np.sin(3 * math.pi * (node // M) / N)
    cx, cy = math.cos(2 * math.pi / N), math.cos(3 * math.pi / N)
    lam = (8 - 2 * cx - 2 * cy - 4 * cx * cy) / 3
    for res in (orc.tfqmr(A, v, 1e-12, 50), orc.bicg(A, v, 1e-12, 50)):
        assert res.status == 0 and res.iters == 1
        assert np.max(np.abs(res.x - v / lam)) <= 1e-12 * np.max(np.abs(v / lam))


def test_bicg_tfqmr_breakdown_and_limits(orc):
    # r.(A D^-1 r) = 0 at the start: both methods break down before a step
    B = orc.assemble(2, np.array([0, 0, 1, 1], np.int32), np.array([0, 1, 0, 1], np.int32),
                     np.array([1.0, -3.0, 1.0, 1.0]))
    b = np.array([1.0, 1.0])
    for res in (orc.bicg(B, b, 1e-10, 10), orc.tfqmr(B, b, 1e-10, 10)):
        assert res.status == -6 and res.iters == 0
    # zero diagonal
    Z = orc.assemble(2, np.array([0, 1], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    assert orc.bicg(Z, b, 1e-10).status == -4 and orc.tfqmr(Z, b, 1e-10).status == -4
    # limits and the zero right-hand side
    probs, bs = W.config6(nsys=1, lo=10, hi=10, seed=8)
    A = orc.assemble(probs[0].n, probs[0].i, probs[0].j, probs[0].v)
    g = orc.bicg(A, bs[0], 1e-14, 4)
    t = orc.tfqmr(A, bs[0], 1e-14, 5)
    assert (g.status, g.iters) == (-5, 4) and (t.status, t.iters) == (-5, 5)
    for res in (orc.bicg(A, np.zeros(A.n), 1e-8), orc.tfqmr(A, np.zeros(A.n), 1e-8)):
        assert res.status == 0 and res.iters == 0 and np.all(res.x == 0)


def test_tfqmr_success_means_true_residual_within_tolerance(orc):
    """On this convection-dominated system the first TFQMR cycle ends on its
    bound with the true residual above the tolerance; the returned x must
    still meet the tolerance in an independent residual."""
    probs, bs = W.config6()
    p, b = probs[20], bs[20]
    A = orc.assemble(p.n, p.i, p.j, p.v)
    t = orc.tfqmr(A, b, 1e-8)
    keep = (p.i >= 0) & (p.j >= 0)
    M = sp.coo_matrix((p.v[keep], (p.i[keep], p.j[keep])), shape=(p.n, p.n)).tocsr()
    assert t.status == 0
    assert np.linalg.norm(b - M @ t.x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-9)
    # a single cycle (restarts impossible: the limit stops at the first pass)
    first = orc.tfqmr(A, b, 1e-8, 470)
    assert first.relres > 1e-8


# ----------------------------------------------------------- L-BFGS H_k g

def explicit_bfgs(S, Y, h0):
    """H_k from diag(h0) by the BFGS update with each pair, oldest first:
    H <- (I - r s y^T) H (I - r y s^T) + r s s^T, r = 1 / s.y."""
    n, m = S.shape
    H = np.diag(h0)
    for j in range(m):
        s, y = S[:, j], Y[:, j]
        r = 1.0 / (s @ y)
        V = np.eye(n) - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return H


@pytest.mark.parametrize("n,m,seed", [(40, 0, 1), (40, 1, 2), (40, 5, 3), (60, 12, 4), (25, 25, 5)])
def test_lbfgs_forms_match_the_explicit_bfgs_matrix(orc, n, m, seed):
    S, Y, g, h0 = W.lbfgs_history(n, m, seed)
    if m:
        assert np.all(np.einsum("ij,ij->j", S, Y) > 0)
    Hg = explicit_bfgs(S, Y, h0) @ g
    for p in (orc.lbfgs_recursive(S, Y, g, h0), orc.lbfgs_dense(S, Y, g, h0)):
        assert np.linalg.norm(p - Hg) <= 1e-12 * np.linalg.norm(Hg)


def test_lbfgs_secant_condition_and_symmetry(orc):
    """H_k y_newest = s_newest exactly in exact arithmetic, and H_k is
    symmetric: a.(H b) = b.(H a)."""
    S, Y, g, h0 = W.lbfgs_history(80, 7, 6)
    for f in (orc.lbfgs_recursive, orc.lbfgs_dense):
        p = f(S, Y, Y[:, -1], h0)
        assert np.linalg.norm(p - S[:, -1]) <= 1e-12 * np.linalg.norm(S[:, -1])
        a, b = np.random.default_rng(7).standard_normal((2, 80))
        assert abs(a @ f(S, Y, b, h0) - b @ f(S, Y, a, h0)) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(b) * 10


def test_lbfgs_listing_reading(orc):
    """With y_j instead of s_j in the second loop (as the paper's listing
    prints it) the result is not H_k g; with s_j it is."""
    S, Y, g, h0 = W.lbfgs_history(30, 4, 8)
    m = S.shape[1]
    q = g.copy()
    alpha = np.zeros(m)
    for j in range(m - 1, -1, -1):
        alpha[j] = (S[:, j] @ q) / (S[:, j] @ Y[:, j])
        q = q - alpha[j] * Y[:, j]
    p = h0 * q
    for j in range(m):
        beta = (Y[:, j] @ p) / (S[:, j] @ Y[:, j])
        p = p + (alpha[j] - beta) * Y[:, j]
    Hg = explicit_bfgs(S, Y, h0) @ g
    assert np.linalg.norm(p - Hg) > 1e-3 * np.linalg.norm(Hg)
    assert np.linalg.norm(orc.lbfgs_recursive(S, Y, g, h0) - Hg) <= 1e-12 * np.linalg.norm(Hg)
