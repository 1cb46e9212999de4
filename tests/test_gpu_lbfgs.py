"""GPU limited-memory BFGS product (intermediate dense form) against the
oracle's two-loop and dense forms."""
import numpy as np
import pytest
import torch

from paper_2406_08646_amd import workloads as W
from gpu_util import dev, host, require_gpu

pytestmark = pytest.mark.gpu


def tol(n):
    """Rounding bound of the dot products of length n (about n eps), twice."""
    return max(1e-12, 2.2e-16 * n)


def pairs_in_use(S, Y, k, m):
    """The oracle's view after k updates with pairs 0..k-1: the last
    min(k, m) of them, oldest first."""
    lo = max(0, k - m)
    return S[:, lo:k], Y[:, lo:k]


@pytest.mark.parametrize("n,m,pushes", [(3000, 5, 12), (777, 1, 3), (2048, 9, 20),
                                        (1500, 33, 40), (5000, 64, 70)])
def test_lbfgs_history_and_product(orc, n, m, pushes):
    spx = require_gpu()
    S, Y, g, h0 = W.lbfgs_history(n, pushes, seed=30 + m)
    L = spx.lbfgs_create(n, m)
    gd, h0d = dev(g), dev(h0)
    # empty history: p = h0 g, exactly
    assert np.array_equal(host(L.apply(gd, h0d)), h0 * g)
    assert np.array_equal(host(L.apply(gd)), g)
    for k in range(1, pushes + 1):
        L.update(dev(np.ascontiguousarray(S[:, k - 1])), dev(np.ascontiguousarray(Y[:, k - 1])))
        assert L.count == min(k, m)
        Sk, Yk = pairs_in_use(S, Y, k, m)
        for h in (h0, None):
            ref = orc.lbfgs_dense(Sk, Yk, g, h0 if h is not None else np.ones(n))
            p = host(L.apply(gd, h0d if h is not None else None))
            err = np.linalg.norm(p - ref) / np.linalg.norm(ref)
            assert err <= tol(n), (k, err)
    L.reset()
    assert L.count == 0
    assert np.array_equal(host(L.apply(gd, h0d)), h0 * g)


def test_lbfgs_secant_condition_on_device(orc):
    spx = require_gpu()
    n, m = 4000, 6
    S, Y, g, h0 = W.lbfgs_history(n, m, seed=40)
    L = spx.lbfgs_create(n, m)
    for j in range(m):
        L.update(dev(np.ascontiguousarray(S[:, j])), dev(np.ascontiguousarray(Y[:, j])))
    p = host(L.apply(dev(np.ascontiguousarray(Y[:, -1])), dev(h0)))
    assert np.linalg.norm(p - S[:, -1]) <= tol(n) * np.linalg.norm(S[:, -1])


def test_lbfgs_argument_errors():
    spx = require_gpu()
    with pytest.raises(spx.SpxError):
        spx.lbfgs_create(10, 0)
    with pytest.raises(spx.SpxError):
        spx.lbfgs_create(10, 65)
    L = spx.lbfgs_create(10, 2)
    g = dev(np.ones(10))
    with pytest.raises(spx.SpxError):
        L.apply(g, p=g)


@pytest.mark.timeout(600)
def test_lbfgs_full_size(orc):
    """n = 10^7, m = 50 (a 4 GB history per factor): after m updates the
    product matches the oracle's two-loop recursion."""
    spx = require_gpu()
    n, m = 10_000_000, 50
    print("lbfgs full size: generating", flush=True)
    S, Y, g, h0 = W.lbfgs_history(n, m, seed=41)
    L = spx.lbfgs_create(n, m)
    for j in range(m):
        L.update(dev(np.ascontiguousarray(S[:, j])), dev(np.ascontiguousarray(Y[:, j])))
    p = host(L.apply(dev(g), dev(h0)))
    print("lbfgs full size: oracle", flush=True)
    ref = orc.lbfgs_recursive(S, Y, g, h0)
    err = np.linalg.norm(p - ref) / np.linalg.norm(ref)
    print(f"lbfgs n={n} m={m}: relative difference {err:.3e}", flush=True)
    assert err <= tol(n)


def test_lbfgs_unaligned_vectors(orc):
    """g, h0 and p 8 bytes off a 16-byte boundary take the one-row-per-thread
    passes; the product matches the aligned call and the oracle."""
    spx = require_gpu()
    n, m = 4096, 20
    S, Y, g, h0 = W.lbfgs_history(n, m, seed=42)
    L = spx.lbfgs_create(n, m)
    for j in range(m):
        L.update(dev(np.ascontiguousarray(S[:, j])), dev(np.ascontiguousarray(Y[:, j])))
    p_al = host(L.apply(dev(g), dev(h0)))
    bufs = [torch.zeros(n + 1, dtype=torch.float64, device="cuda") for _ in range(3)]
    bufs[0][1:] = dev(g)
    bufs[1][1:] = dev(h0)
    gu, hu, pu = (b[1:] for b in bufs)
    assert gu.data_ptr() % 16 == 8
    L.apply(gu, hu, p=pu)
    p_un = host(pu)
    ref = orc.lbfgs_dense(S, Y, g, h0)
    for p in (p_al, p_un):
        assert np.linalg.norm(p - ref) <= tol(n) * np.linalg.norm(ref)
    assert np.linalg.norm(p_un - p_al) <= tol(n) * np.linalg.norm(ref)


@pytest.mark.parametrize("n,m,pushes,offset", [(3000, 5, 12, 0), (2049, 7, 10, 0), (4096, 20, 24, 0),
                                               (4096, 20, 6, 1), (1000, 64, 3, 0)])
def test_lbfgs_update_apply_same_bits(orc, n, m, pushes, offset):
    """The fused step equals update then apply bit for bit, through ring
    wrap-around, for even n (two rows per thread), odd n (one), and vectors
    off a 16-byte boundary (taken unfused); and matches the oracle."""
    spx = require_gpu()
    S, Y, g, h0 = W.lbfgs_history(n, pushes, seed=60 + m)
    A, B = spx.lbfgs_create(n, m), spx.lbfgs_create(n, m)
    bufs = [torch.zeros(n + offset, dtype=torch.float64, device="cuda") for _ in range(3)]
    bufs[0][offset:] = dev(g)
    bufs[1][offset:] = dev(h0)
    gd, h0d, pd = (b[offset:] for b in bufs)
    for k in range(1, pushes + 1):
        s, y = dev(np.ascontiguousarray(S[:, k - 1])), dev(np.ascontiguousarray(Y[:, k - 1]))
        hk = h0d if k % 3 else None  # every third step with H0 = I
        A.update(s, y)
        pa = host(A.apply(gd, hk))
        B.update_apply(s, y, gd, hk, p=pd)
        pb = host(pd)
        assert A.count == B.count == min(k, m)
        assert np.array_equal(pa.view(np.int64), pb.view(np.int64)), k
        Sk, Yk = pairs_in_use(S, Y, k, m)
        ref = orc.lbfgs_dense(Sk, Yk, g, h0 if hk is not None else np.ones(n))
        assert np.linalg.norm(pb - ref) <= tol(n) * np.linalg.norm(ref), k
    # the products the update stored serve later plain applies
    assert np.array_equal(host(A.apply(gd)).view(np.int64), host(B.apply(gd)).view(np.int64))
    with pytest.raises(spx.SpxError):
        B.update_apply(s, y, gd, p=gd)
