"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def to_dev(torch, *arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrays]


def col_relerr(X, Y):
    """max over RHS columns of ||X - Y||_2 / ||Y||_2 (arrays of shape (N, M, R))."""
    R = Y.shape[2]
    d = (X - Y).reshape(-1, R)
    n = np.linalg.norm(Y.reshape(-1, R), axis=0)
    return float(np.max(np.linalg.norm(d, axis=0) / np.where(n > 0, n, 1.0)))


def assert_parity(X, Xo, tol=1e-10):
    """Element-by-element comparison scaled by the column norm, plus the column
    relative error bound."""
    assert X.shape == Xo.shape
    assert np.all(np.isfinite(X))
    err = col_relerr(X, Xo)
    assert err <= tol, f"relative error {err:.3e} > {tol:.1e}"
    scale = np.max(np.abs(Xo), axis=(0, 1), keepdims=True)
    assert np.all(np.abs(X - Xo) <= tol * np.maximum(scale, 1e-300)), "element outside tolerance"
    return err
