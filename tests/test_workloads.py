"""Invariants of the seeded input generators (CPU)."""
import numpy as np

from paper_2406_08646_amd import workloads as W


def test_config_sizes():
    prob, x, b = W.config1()
    assert prob.n == 4096 and prob.ncoo == 63 * 63 * 16 and x.shape == b.shape == (4096,)
    assert np.all((-1 <= x) & (x <= 1))
    p = W.q1_poisson(5, 3)
    assert p.n == 216 and p.ncoo == 125 * 64 and p.i.dtype == np.int32
    probs, bs = W.config4()
    assert len(probs) == 64
    for pr, bb in zip(probs, bs):
        L = pr.grid
        assert 32 <= L <= 512 and pr.n == L * L and pr.ncoo == 8 * L * L - 4 * L
        assert bb.shape == (pr.n,)


def test_element_contiguity_and_orderings():
    N = 3
    p = W.q1_poisson(N, 2)
    e, a, b = 4, 2, 1  # element (1,1), local node (0,1), (1,0)
    k = 16 * e + 4 * a + b
    M = N + 1
    assert p.i[k] == (1 + 0) + M * (1 + 1) and p.j[k] == (1 + 1) + M * (1 + 0)
    # every element's 16 triplets are contiguous and couple its 4 corners
    for e in range(N * N):
        blk = slice(16 * e, 16 * (e + 1))
        assert len(set(p.i[blk])) == 4 and set(p.i[blk]) == set(p.j[blk])


def test_dirichlet_elimination_values():
    N = 4
    p = W.q1_poisson(N, 2, kappa=np.full(16, 2.0))
    M = N + 1
    node = np.arange(p.n)
    bnd = (node % M == 0) | (node % M == N) | (node // M == 0) | (node // M == N)
    touch = bnd[p.i] | bnd[p.j]
    diag_b = bnd[p.i] & (p.i == p.j)
    assert np.all(p.v[touch & ~diag_b] == 0.0)
    assert np.all(np.isin(p.v[diag_b], [1.0, 0.5]))
    assert np.all(p.dv_dlogk[touch] == 0.0)
    assert np.array_equal(p.dv_dlogk[~touch], p.v[~touch])


def test_element_coefficient_split_reproduces_stream():
    N = 8
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(N * N)
    one = W.q1_poisson(N, 2, kappa=np.ones(N * N))
    base, w = one.v - one.dv_dlogk, one.dv_dlogk
    v = base + np.repeat(np.exp(theta), 16) * w
    ref = W.q1_poisson(N, 2, kappa=np.exp(theta))
    assert np.array_equal(v.view(np.uint64), ref.v.view(np.uint64))


def test_five_point_symmetric_stream():
    rng = np.random.default_rng(1)
    L = 7
    p = W.five_point_system(L, rng.random(42), rng.random(42), rng.random(28))
    D = np.zeros((p.n, p.n))
    np.add.at(D, (p.i, p.j), p.v)
    assert np.allclose(D, D.T) and np.all(np.linalg.eigvalsh(D) > 0)


def test_fd_sample_is_reproducible():
    a = W.fd_sample(256, 20)
    assert np.array_equal(a, W.fd_sample(256, 20)) and len(np.unique(a)) == 20
