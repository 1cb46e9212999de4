"""Seeded synthetic inputs for the COO assembly / SpMV / CG path.

This module only *generates data*: COO index/value triplets of finite-element
and finite-volume model problems, right-hand sides, starting vectors and
random parameters.  It performs none of the method's arithmetic (no sorting,
no summation of duplicates, no products with the assembled matrix, no
solves), so both the GPU path and the CPU oracle can consume its output
without sharing any of the computation under test.

Layout conventions (paper Sec. 5, "Portable matrix assembly on GPUs",
finite-element usage paragraph): the triplets of one element matrix are
stored contiguously, elements follow each other in lexicographic order, and
all elements have the same size, so the offset of element ``e`` in ``v`` is
``e * nloc**2``.

Orderings (x fastest everywhere):
  * element  e = ex + N*(ey + N*ez)
  * node     g = ix + M*(iy + M*iz),  M = N + 1
  * local    a = dx + 2*dy (+ 4*dz)
  * triplet  k = e*nloc**2 + a*nloc + b,   (i[k], j[k]) = (g(e,a), g(e,b))

Dirichlet rows are eliminated symmetrically *inside* the COO stream so the
pattern keeps every triplet: for a boundary node g_a the diagonal
contribution of each touching element is 1/mult(g_a) (mult = number of
elements sharing that node, a power of two, so the assembled diagonal is
exactly 1.0), every other triplet that touches a boundary node carries 0.0,
and interior-interior pairs carry kappa_e * h**(d-2) * Kref[a, b].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "CooProblem",
    "q1_reference_stiffness",
    "q1_poisson",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "spmm_rhs",
    "fd_sample",
    "random_coo",
    "periodic_tridiag_jacobian",
    "five_point_system",
]


@dataclasses.dataclass
class CooProblem:
    """A COO triplet stream ``(i, j, v)`` of an ``n x n`` matrix.

    ``dv_dlogk`` (optional) holds d v[k] / d theta_e for the element that
    emitted triplet ``k`` when the element coefficient is kappa_e =
    exp(theta_e): it equals ``v[k]`` for interior-interior pairs and 0.0 for
    the Dirichlet-elimination triplets.
    """

    n: int
    i: np.ndarray  # int32[ncoo]
    j: np.ndarray  # int32[ncoo]
    v: np.ndarray  # float64[ncoo]
    nelem: int = 0
    nloc: int = 0
    grid: int = 0
    dim: int = 0
    dv_dlogk: Optional[np.ndarray] = None

    @property
    def ncoo(self) -> int:
        return int(self.i.shape[0])


# ---------------------------------------------------------------------------
# Q1 element matrices (tensor products of the 1-D P1 stiffness and mass).
# ---------------------------------------------------------------------------

def q1_reference_stiffness(dim: int) -> np.ndarray:
    """Reference Laplacian element matrix of the Q1 element on a unit cube
    (2-D: bilinear square, 3-D: trilinear hexahedron), local nodes numbered
    a = dx + 2 dy (+ 4 dz).  Entries depend only on how many coordinates
    two local nodes differ in:

      2-D: 0 -> 2/3, 1 -> -1/6, 2 -> -1/3
      3-D: 0 -> 1/3, 1 -> 0,    2 -> -1/12, 3 -> -1/12

    The 3-D matrix must be multiplied by h to give the element matrix of a
    cube of side h; the 2-D one is scale free.  Literals are the correctly
    rounded quotients.
    """
    if dim == 2:
        table = {0: 2.0 / 3.0, 1: -1.0 / 6.0, 2: -1.0 / 3.0}
    elif dim == 3:
        table = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}
    else:
        raise ValueError("dim must be 2 or 3")
    nloc = 1 << dim
    K = np.empty((nloc, nloc), dtype=np.float64)
    for a in range(nloc):
        for b in range(nloc):
            K[a, b] = table[bin(a ^ b).count("1")]
    return K


def q1_poisson(N: int, dim: int, kappa: Optional[np.ndarray] = None) -> CooProblem:
    """COO stream of the Q1 Poisson operator on the unit square/cube with N
    elements per side, per-element coefficient ``kappa`` (default 1) and
    Dirichlet nodes eliminated symmetrically as described in the module
    docstring."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    M = N + 1
    n = M**dim
    nloc = 1 << dim
    nelem = N**dim
    h = 1.0 / N
    Kref = q1_reference_stiffness(dim)
    Kh = Kref * h if dim == 3 else Kref.copy()

    e = np.arange(nelem, dtype=np.int64)
    coords = []
    rem = e
    for _ in range(dim):
        coords.append(rem % N)
        rem = rem // N
    loc = np.arange(nloc)
    doff = [(loc >> d) & 1 for d in range(dim)]

    # node coordinates (nelem, nloc) per dimension, global node ids, boundary flags
    g = np.zeros((nelem, nloc), dtype=np.int64)
    bnd = np.zeros((nelem, nloc), dtype=bool)
    mult = np.ones((nelem, nloc), dtype=np.int64)
    stride = 1
    for d in range(dim):
        c = coords[d][:, None] + doff[d][None, :]
        g += c * stride
        on = (c == 0) | (c == N)
        bnd |= on
        mult *= np.where(on, 1, 2)
        stride *= M
    del coords

    if n > np.iinfo(np.int32).max:
        raise ValueError("grid too large for int32 indices")
    gi = g.astype(np.int32)
    del g
    i = np.ascontiguousarray(np.broadcast_to(gi[:, :, None], (nelem, nloc, nloc))).reshape(-1)
    j = np.ascontiguousarray(np.broadcast_to(gi[:, None, :], (nelem, nloc, nloc))).reshape(-1)
    del gi

    if kappa is None:
        v = np.broadcast_to(Kh[None, :, :], (nelem, nloc, nloc)).copy()
    else:
        kappa = np.asarray(kappa, dtype=np.float64)
        if kappa.shape != (nelem,):
            raise ValueError("kappa must have one entry per element")
        v = kappa[:, None, None] * Kh[None, :, :]
    interior = ~(bnd[:, :, None] | bnd[:, None, :])
    dv = np.where(interior, v, 0.0).reshape(-1) if kappa is not None else None
    v[~interior] = 0.0
    diag = np.arange(nloc)
    vd = v[:, diag, diag]  # (nelem, nloc) copy
    vd = np.where(bnd, 1.0 / mult, vd)
    v[:, diag, diag] = vd
    del interior, bnd, mult, vd
    return CooProblem(n=n, i=i, j=j, v=v.reshape(-1), nelem=nelem, nloc=nloc,
                      grid=N, dim=dim, dv_dlogk=dv)


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

def config1():
    """2-D Q1 Poisson, 63 x 63 elements (4096 nodes), kappa = 1; x then b
    ~ U[-1, 1] from seed 0.  CG tolerance 1e-8."""
    prob = q1_poisson(63, 2)
    rng = np.random.default_rng(0)
    x = rng.uniform(-1.0, 1.0, prob.n)
    b = rng.uniform(-1.0, 1.0, prob.n)
    return prob, x, b


def config2(N: int = 127):
    """3-D Q1 Poisson, N^3 elements ((N+1)^3 nodes, 64 triplets each),
    kappa = 1, h = 1/N; x then b ~ U[-1, 1] from seed 0.  CG tolerance
    1e-10.  N = 127 is the full-size workload; smaller N keep the same
    structure."""
    prob = q1_poisson(N, 3)
    rng = np.random.default_rng(0)
    x = rng.uniform(-1.0, 1.0, prob.n)
    b = rng.uniform(-1.0, 1.0, prob.n)
    return prob, x, b


def config3(N: int = 127):
    """Same mesh as :func:`config2` with log-normal element diffusivity
    kappa_e = exp(z_e), z ~ N(0, 1) (sigma = 1, no mean shift) from seed 1,
    followed by b ~ U[-1, 1] from the same generator."""
    rng = np.random.default_rng(1)
    z = rng.standard_normal(N**3)
    prob = q1_poisson(N, 3, kappa=np.exp(z))
    b = rng.uniform(-1.0, 1.0, prob.n)
    return prob, b


def five_point_system(L: int, c_h: np.ndarray, c_v: np.ndarray, c_b: np.ndarray) -> CooProblem:
    """COO stream of a 2-D 5-point finite-volume diffusion operator on an
    L x L cell grid with Dirichlet exterior.  Unknown p = x + L*y.

    ``c_h`` ((L-1)*L): coefficients of the edges (x,y)-(x+1,y), y-major.
    ``c_v`` (L*(L-1)): coefficients of the edges (x,y)-(x,y+1), y-major.
    ``c_b`` (4L): boundary faces, in the order left (y = 0..L-1), right,
    bottom (x = 0..L-1), top.
    An interior edge (p,q,c) emits (p,p,+c),(p,q,-c),(q,p,-c),(q,q,+c); a
    boundary face at p emits (p,p,+c)."""
    ys, xs = np.meshgrid(np.arange(L), np.arange(L - 1), indexing="ij")
    hp = (xs + L * ys).reshape(-1)
    hq = hp + 1
    ys, xs = np.meshgrid(np.arange(L - 1), np.arange(L), indexing="ij")
    vp = (xs + L * ys).reshape(-1)
    vq = vp + L
    p = np.concatenate([hp, vp])
    q = np.concatenate([hq, vq])
    c = np.concatenate([np.asarray(c_h, np.float64), np.asarray(c_v, np.float64)])
    ii = np.stack([p, p, q, q], axis=1).reshape(-1)
    jj = np.stack([p, q, p, q], axis=1).reshape(-1)
    vv = np.stack([c, -c, -c, c], axis=1).reshape(-1)
    r = np.arange(L)
    bp = np.concatenate([r * L, r * L + (L - 1), r, r + L * (L - 1)])
    ii = np.concatenate([ii, bp]).astype(np.int32)
    jj = np.concatenate([jj, bp]).astype(np.int32)
    vv = np.concatenate([vv, np.asarray(c_b, np.float64)])
    return CooProblem(n=L * L, i=ii, j=jj, v=vv, grid=L, dim=2)


def config4(nsys: int = 64, lo: int = 32, hi: int = 512, sigma: float = 0.5, seed: int = 3):
    """Batch of ``nsys`` 5-point variable-coefficient diffusion systems.
    Draw order from ``default_rng(seed)``: the sides round(exp(U[ln lo,
    ln hi])) of all systems; then, system by system, standard normals z for
    the horizontal, vertical and boundary edges (coefficient exp(sigma*z));
    then, system by system, b ~ U[-1, 1].  CG tolerance 1e-8."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), nsys))).astype(np.int64)
    probs: List[CooProblem] = []
    for L in sides:
        L = int(L)
        z = rng.standard_normal(2 * L * (L - 1) + 4 * L)
        c = np.exp(sigma * z)
        nh = L * (L - 1)
        probs.append(five_point_system(L, c[:nh], c[nh:2 * nh], c[2 * nh:]))
    bs = [rng.uniform(-1.0, 1.0, p.n) for p in probs]
    return probs, bs


def convection_diffusion_system(L: int, c_h: np.ndarray, c_v: np.ndarray, c_b: np.ndarray,
                                wx: float, wy: float) -> CooProblem:
    """The 5-point diffusion stream of ``five_point_system`` followed by a
    first-order upwind convection stream for the constant velocity (wx, wy)
    on the same cell grid (unit spacing, Dirichlet exterior with value 0).

    Across the face between cells p (upstream) and q (downstream) with
    normal speed w > 0, the flux w*u_p leaves p and enters q: triplets
    (p, p, +w), (q, p, -w).  A boundary face with outflow w at cell p
    emits (p, p, +w); inflow faces carry the zero exterior value and emit
    nothing.  The matrix is an M-matrix and not symmetric unless w = 0."""
    base = five_point_system(L, c_h, c_v, c_b)
    ii, jj, vv = [base.i], [base.j], [base.v]
    ys, xs = np.meshgrid(np.arange(L), np.arange(L - 1), indexing="ij")
    hp = (xs + L * ys).reshape(-1)
    ys, xs = np.meshgrid(np.arange(L - 1), np.arange(L), indexing="ij")
    vp = (xs + L * ys).reshape(-1)
    r = np.arange(L)
    for w, lo, hi, face_lo, face_hi in ((float(wx), hp, hp + 1, r * L, r * L + (L - 1)),
                                        (float(wy), vp, vp + L, r, r + L * (L - 1))):
        if w == 0.0:
            continue
        up, down = (lo, hi) if w > 0 else (hi, lo)
        a = abs(w)
        m = up.shape[0]
        ii.append(np.stack([up, down], axis=1).reshape(-1))
        jj.append(np.stack([up, up], axis=1).reshape(-1))
        vv.append(np.tile([a, -a], m))
        out = face_hi if w > 0 else face_lo
        ii.append(out)
        jj.append(out)
        vv.append(np.full(L, a))
    return CooProblem(n=L * L, i=np.concatenate(ii).astype(np.int32),
                      j=np.concatenate(jj).astype(np.int32), v=np.concatenate(vv), grid=L, dim=2)


def config6(nsys: int = 64, lo: int = 32, hi: int = 512, sigma: float = 0.5,
            speed: tuple = (0.5, 2.0), seed: int = 5):
    """Non-symmetric batch: ``nsys`` upwind convection-diffusion systems.
    Draw order from ``default_rng(seed)``: the sides round(exp(U[ln lo,
    ln hi])); then, system by system, standard normals z for the horizontal,
    vertical and boundary diffusion edges (coefficient exp(sigma*z)) and the
    velocity (speed ~ U[speed], angle ~ U[0, 2 pi)); then, system by system,
    b ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), nsys))).astype(np.int64)
    probs: List[CooProblem] = []
    for L in sides:
        L = int(L)
        z = rng.standard_normal(2 * L * (L - 1) + 4 * L)
        c = np.exp(sigma * z)
        sp = rng.uniform(*speed)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        nh = L * (L - 1)
        probs.append(convection_diffusion_system(L, c[:nh], c[nh:2 * nh], c[2 * nh:],
                                                 sp * math.cos(ang), sp * math.sin(ang)))
    bs = [rng.uniform(-1.0, 1.0, p.n) for p in probs]
    return probs, bs


def lbfgs_history(n: int, m: int, seed: int = 6):
    """A limited-memory history for H_k g: S ~ N(0, 1) (n x m, oldest pair
    first), Y = d * S + 0.1 N(0, 1) with a per-row curvature d ~ U[0.5, 2]
    (so s_j . y_j > 0), the gradient g ~ N(0, 1) and a diagonal base
    operator h0 ~ U[0.5, 1.5].  Draw order: d, S, noise, g, h0.  S and Y are
    column-major (each pair contiguous)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 2.0, n)
    S = np.asfortranarray(rng.standard_normal((n, m)))
    Y = np.asfortranarray(d[:, None] * S + 0.1 * rng.standard_normal((n, m)))
    g = rng.standard_normal(n)
    h0 = rng.uniform(0.5, 1.5, n)
    return S, Y, g, h0


def config5(N: int = 256):
    """2-D Q1 Poisson on N x N elements with kappa_e = exp(theta_e), theta ~
    N(0, 1) from seed 2, right-hand side b = 1.  Returns the problem (with
    ``dv_dlogk``), theta, the target problem at theta* = 0 and b."""
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(N * N)
    prob = q1_poisson(N, 2, kappa=np.exp(theta))
    target = q1_poisson(N, 2, kappa=np.ones(N * N))
    b = np.ones(prob.n)
    return prob, theta, target, b


def fd_sample(N: int = 256, count: int = 20):
    """Indices of the theta entries checked by finite differences: drawn
    from ``default_rng(2)`` after theta (without replacement)."""
    rng = np.random.default_rng(2)
    rng.standard_normal(N * N)
    return np.sort(rng.choice(N * N, size=count, replace=False))


def spmm_rhs(n: int, nrhs: int = 16, seed: int = 4) -> np.ndarray:
    """Row-major n x nrhs block of right-hand sides ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (n, nrhs))


# ---------------------------------------------------------------------------
# Generic streams for fuzzing and small worked examples.
# ---------------------------------------------------------------------------

def random_coo(rng: np.random.Generator, n: int, ncoo: int, *, neg_frac: float = 0.1,
               dup_pool: Optional[int] = None, extreme: bool = True) -> CooProblem:
    """Random non-symmetric COO stream with many duplicates, negative
    (ignored) indices, signed zeros and cancellation-heavy magnitudes."""
    if dup_pool is None:
        dup_pool = max(1, ncoo // 3)
    pi = rng.integers(0, n, dup_pool)
    pj = rng.integers(0, n, dup_pool)
    pick = rng.integers(0, dup_pool, ncoo)
    i = pi[pick].astype(np.int32)
    j = pj[pick].astype(np.int32)
    if neg_frac > 0:
        neg = rng.random(ncoo) < neg_frac
        which = rng.integers(0, 3, ncoo)
        i[neg & (which != 1)] = -1 - rng.integers(0, 5, int(np.sum(neg & (which != 1))))
        j[neg & (which != 0)] = -1 - rng.integers(0, 5, int(np.sum(neg & (which != 0))))
    if extreme:
        mant = rng.uniform(-1.0, 1.0, ncoo)
        expo = rng.integers(-60, 61, ncoo)
        v = np.ldexp(mant, expo)
        z = rng.random(ncoo)
        v[z < 0.05] = 0.0
        v[(z >= 0.05) & (z < 0.10)] = -0.0
    else:
        v = rng.uniform(-1.0, 1.0, ncoo)
    return CooProblem(n=n, i=i, j=j, v=v)


def periodic_tridiag_jacobian(n: int, d: float, X: np.ndarray) -> CooProblem:
    """Jacobian of the 1-D periodic residual R_i = d (X_{i-1} - 2 X_i +
    X_{i+1}) + X_i^2 - F_i as three COO triplets per row in the order
    (i,i-1), (i,i), (i,i+1), with values d, -2d + 2 X_i, d (the worked
    Kokkos example of paper Sec. 3, Jacobian callback listing)."""
    r = np.arange(n)
    i = np.repeat(r, 3).astype(np.int32)
    j = np.stack([(r - 1) % n, r, (r + 1) % n], axis=1).reshape(-1).astype(np.int32)
    X = np.asarray(X, np.float64)
    v = np.stack([np.full(n, d), -2.0 * d + 2.0 * X, np.full(n, d)], axis=1).reshape(-1)
    return CooProblem(n=n, i=i, j=j, v=v)
