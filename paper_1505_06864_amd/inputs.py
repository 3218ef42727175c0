"""Seeded synthetic inputs for block-tridiagonal systems.

This module holds input recipes only -- no step of the solver -- and is the
one place both the GPU library's tests/benchmark and the CPU oracle take
their inputs from.  All arrays are numpy float64, row-major:
``A, B, C`` of shape ``(N, M, M)`` (diagonal, sub-diagonal, super-diagonal
blocks of ``B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i``), ``F`` of shape
``(N, M, R)``.  ``B[0]`` and ``C[N-1]`` are drawn (so the random stream does
not depend on the boundary convention) but are not part of the matrix.

Recipes (stand-ins for the paper's workloads, whose matrices are not
published: a 2D-Laplace discretisation with small random fill for its
validation runs, Sec. 6, and the Faddeev boundary-value problem with dense
diagonal and banded off-diagonal blocks, Sec. 7):

* ``diag_dominant``: A_i = U(-1,1)/(4M) + shift*I, B_i, C_i = U(-1,1)/(4M),
  x* ~ N(0,1), F = A x*.  Block diagonally dominant.
* ``faddeev_like``: h = 1/N, S = symmetric Toeplitz band (1, .25, .1, .02),
  K = M^2 * symmetric Toeplitz band (2, -.6, -.3, -.1), v_i = 1 + U(0,1),
  A_i = (2/h^2) S + K + v_i S, B_i = C_i = -S/h^2, F ~ N(0,1).

Draw order with ``numpy.random.default_rng(seed)`` (PCG64): A, then B, then
C, then x* (or F).
"""
import numpy as np


def _band_toeplitz(M, band):
    T = np.zeros((M, M))
    for d, v in enumerate(band):
        idx = np.arange(M - d)
        T[idx, idx + d] = v
        T[idx + d, idx] = v
    return T


def block_matvec(A, B, C, X):
    """F = (block-tridiagonal A) X, used to manufacture right-hand sides."""
    F = np.einsum("nij,njr->nir", A, X)
    if A.shape[0] > 1:
        F[1:] += np.einsum("nij,njr->nir", B[1:], X[:-1])
        F[:-1] += np.einsum("nij,njr->nir", C[:-1], X[1:])
    return F


def diag_dominant(N, M, R, seed, shift=2.0, want_xstar=False):
    rng = np.random.default_rng(seed)
    s = 1.0 / (4.0 * M)
    A = rng.uniform(-1.0, 1.0, size=(N, M, M)) * s
    A += shift * np.eye(M)[None]
    B = rng.uniform(-1.0, 1.0, size=(N, M, M)) * s
    C = rng.uniform(-1.0, 1.0, size=(N, M, M)) * s
    xs = rng.standard_normal((N, M, R))
    F = block_matvec(A, B, C, xs)
    return (A, B, C, F, xs) if want_xstar else (A, B, C, F)


def faddeev_like(N, M, R, seed):
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    S = _band_toeplitz(M, (1.0, 0.25, 0.1, 0.02))
    K = float(M) ** 2 * _band_toeplitz(M, (2.0, -0.6, -0.3, -0.1))
    v = 1.0 + rng.uniform(0.0, 1.0, size=N)
    A = (2.0 / h**2) * S[None] + K[None] + v[:, None, None] * S[None]
    B = np.broadcast_to(-S / h**2, (N, M, M)).copy()
    C = B.copy()
    F = rng.standard_normal((N, M, R))
    return A, B, C, F


# Named workloads: small dense-block case, Faddeev-like banded blocks, large
# dense-block case (shift 1.5).
def cfg_small(R=1, seed=0):
    return diag_dominant(64, 16, R, seed, shift=2.0)


def cfg_faddeev(N=2048, M=128, R=4, seed=1):
    return faddeev_like(N, M, R, seed)


def cfg_large(R=1, seed=2, N=4096, M=256):
    return diag_dominant(N, M, R, seed, shift=1.5)


# Batched uneven systems: (N, M, R) per system drawn with numpy's PCG64 from
# `seed` (N ~ U{32..1024}, M from {32, 64, 128, 192}, R from {1, 8, 32}),
# each system drawn with the small workload's recipe (diag_dominant, shift
# 2) from its own seed 3000 + s.
def uneven_specs(count=512, seed=3, n_range=(32, 1024), blocks=(32, 64, 128, 192), rhs=(1, 8, 32)):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(n_range[0], n_range[1] + 1)), int(rng.choice(blocks)), int(rng.choice(rhs)))
            for _ in range(count)]


def uneven_system(spec, s):
    N, M, R = spec
    return diag_dominant(N, M, R, seed=3000 + s, shift=2.0)


def diag_dominant_device(N, M, R, seed, shift=2.0, device="cuda", out=None):
    """The diag_dominant recipe drawn on the device with torch's generator
    (a different random stream from the numpy recipe; for inputs too large
    to draw on the host): A_i = U(-1,1)/(4M) + shift I, B_i, C_i =
    U(-1,1)/(4M), F ~ N(0, 1).  `out` = optional (A, B, C) tensors to fill."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    s = 1.0 / (4.0 * M)
    arrs = out or tuple(torch.empty((N, M, M), dtype=torch.float64, device=device) for _ in range(3))
    for a in arrs:
        a.uniform_(-s, s, generator=g)
    arrs[0].diagonal(dim1=1, dim2=2).add_(shift)
    F = torch.empty((N, M, R), dtype=torch.float64, device=device).normal_(generator=g)
    return (*arrs, F)
