"""Differentiation of u = A(theta)^-1 b through the COO assembly against the
oracle gradient and central finite differences with direct solves."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from paper_2406_08646_amd import autograd as AG, workloads as W
from gpu_util import dev, host, require_gpu

pytestmark = pytest.mark.gpu


def element_parts(N):
    """base + exp(theta_e) w reproduces the kappa = exp(theta) stream."""
    one = W.q1_poisson(N, 2, kappa=np.ones(N * N))
    w = one.dv_dlogk
    base = one.v - w
    return one, base, w


def oracle_gradient(orc, N, theta, b, ustar):
    prob = W.q1_poisson(N, 2, kappa=np.exp(theta))
    A = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    u = orc.pcg(A, b, 1e-13).x
    lam = orc.pcg(A, u - ustar, 1e-13).x  # A symmetric
    gv = orc.coo_grad(prob.i, prob.j, lam, u)
    return orc.block_reduce(gv, prob.dv_dlogk, 16), u


def direct(N, theta, b):
    prob = W.q1_poisson(N, 2, kappa=np.exp(theta))
    keep = (prob.i >= 0) & (prob.j >= 0)
    S = sp.coo_matrix((prob.v[keep], (prob.i[keep], prob.j[keep])), shape=(prob.n, prob.n)).tocsc()
    return spla.spsolve(S, b)


@pytest.mark.parametrize("N", [16, 64])
def test_gradient_matches_oracle_and_fd(orc, N):
    spx = require_gpu()
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(N * N)
    one, base, w = element_parts(N)
    b = np.ones(one.n)
    ustar = direct(N, np.zeros(N * N), b)
    A = spx.coo_preallocate(one.n, dev(one.i), dev(one.j))
    th = dev(theta).requires_grad_(True)
    u = AG.element_coefficient_solve(th, dev(b), A, dev(base), dev(w), 16, rtol=1e-13)
    loss = 0.5 * torch.sum((u - dev(ustar)) ** 2)
    loss.backward()
    g = host(th.grad)
    g_ref, u_ref = oracle_gradient(orc, N, theta, b, ustar)
    assert np.linalg.norm(host(u) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)
    idx = np.sort(rng.choice(N * N, 20, replace=False))
    h = 1e-4
    fd = []
    for e in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h
        tm[e] -= h
        lp = 0.5 * np.sum((direct(N, tp, b) - ustar) ** 2)
        lm = 0.5 * np.sum((direct(N, tm, b) - ustar) ** 2)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    err = np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd)
    print(f"N={N}: |grad - fd| / |fd| = {err:.2e}", flush=True)
    assert err <= 1e-6


def test_generic_coo_solve_gradient(orc):
    spx = require_gpu()
    prob, theta, _, b = W.config5(N=12)
    A = spx.coo_preallocate(prob.n, dev(prob.i), dev(prob.j))
    v = dev(prob.v).requires_grad_(True)
    bt = dev(b).requires_grad_(True)
    u = AG.coo_solve(v, bt, A, rtol=1e-13)
    gu = np.random.default_rng(3).uniform(-1, 1, prob.n)
    (u * dev(gu)).sum().backward()
    R = orc.assemble(prob.n, prob.i, prob.j, prob.v)
    uo = orc.pcg(R, b, 1e-13).x
    lam = orc.pcg(R, gu, 1e-13).x
    gv = orc.coo_grad(prob.i, prob.j, lam, uo)
    assert np.linalg.norm(host(v.grad) - gv) <= 1e-9 * np.linalg.norm(gv)
    assert np.linalg.norm(host(bt.grad) - lam) <= 1e-9 * np.linalg.norm(lam)


@pytest.mark.timeout(900)
def test_gradient_full_config(orc):
    """256 x 256 elements, theta ~ N(0,1) (seed 2), b = 1, rtol 1e-12:
    gradient against central differences (direct solves) on the 20 sampled
    theta entries and against the oracle gradient."""
    spx = require_gpu()
    N = 256
    prob, theta, target, b = W.config5(N)
    one, base, w = element_parts(N)
    ustar = direct(N, np.zeros(N * N), b)
    A = spx.coo_preallocate(one.n, dev(one.i), dev(one.j))
    th = dev(theta).requires_grad_(True)
    u = AG.element_coefficient_solve(th, dev(b), A, dev(base), dev(w), 16, rtol=1e-12)
    loss = 0.5 * torch.sum((u - dev(ustar)) ** 2)
    loss.backward()
    g = host(th.grad)
    idx = W.fd_sample(N, 20)
    h = 1e-4
    fd = []
    for e in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h
        tm[e] -= h
        fd.append((0.5 * np.sum((direct(N, tp, b) - ustar) ** 2)
                   - 0.5 * np.sum((direct(N, tm, b) - ustar) ** 2)) / (2 * h))
    fd = np.array(fd)
    err = np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd)
    print(f"full config: |grad - fd| / |fd| on 20 entries = {err:.2e}", flush=True)
    assert err <= 1e-6
    g_ref, _ = oracle_gradient(orc, N, theta, b, ustar)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"full config: |grad - oracle| / |oracle| = {rel:.2e}", flush=True)
    assert rel <= 1e-6
