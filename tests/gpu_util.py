"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_08646_amd import spx

    spx.load_library()  # raises if the HIP library is missing
    return spx


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def assemble(spx, prob):
    A = spx.coo_preallocate(prob.n, dev(prob.i), dev(prob.j))
    A.set_values_coo(dev(prob.v))
    return A


def csr_equal(orc_A, rowptr, col, val):
    assert np.array_equal(rowptr, orc_A.rowptr)
    assert np.array_equal(col, orc_A.col)
    assert np.array_equal(bits(val), bits(orc_A.val))


def spmv_within(y, ref, scale, tol=1e-12):
    """Componentwise |y - ref| <= tol (|A||x|) + 1e-300."""
    err = np.abs(y - ref)
    bound = tol * scale + 1e-300
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]])
