"""FP64 CPU oracle for the decomposition method (DM) of arXiv:1505.06864.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library (``paper_1505_06864_amd``) and imports nothing
from it; the two meet only in the seeded input generators.

Notation: ``B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i`` with A diagonal,
B sub-diagonal and C super-diagonal ``M x M`` blocks (the paper's C, A and
B of its problem statement, Sec. 2 Eq. eq01), ``N`` block rows, ``R``
right-hand-side columns, ``P`` subsystems.  Arrays are numpy float64,
``A, B, C`` of shape ``(N, M, M)``, ``F, X`` of shape ``(N, M, R)``.

Functions and the passage each follows:
  ta_solve       Thomas algorithm, Sec. 3 (explicit inverses G_i, Sec. 4).
  dm_solve       DM, Sec. 2 (Eqs. e220-e232, endSolution); recursion on the
                 coupling system, Sec. 4.2 (Eq. DMrec1); recursion into the
                 subsystems (J sub-subsystems, Sec. 4.2.2) and both.
  gepp_solve     dense Gaussian elimination with partial pivoting.
  residual       ||F - A X||_2 / ||F||_2 per column.
  partition      equal-split separators (Sec. 2 and Sec. 5).
  balanced_partition
                 first and last subsystems alpha and beta times the middle
                 ones (Sec. 5.1, second case of the speedup analysis, Eq. SpeedupMPNk).
  default_m      coupling-system subsystem count (Eq. SuppMatrM).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class Counter(ctypes.Structure):
    """Block operations in the paper's units (Sec. 4)."""
    _fields_ = [("inv", ctypes.c_longlong), ("mm", ctypes.c_longlong), ("mr", ctypes.c_longlong)]

    def as_dict(self):
        return {"inv": self.inv, "mm": self.mm, "mr": self.mr}


class _Aux(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("D", "E", "ZL", "ZR", "y", "z", "Hd", "Hb", "Hc", "fhat", "h")]


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_inverse.argtypes = [ctypes.c_int, dp, dp]
        L.or_partition.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        L.or_default_m.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_ta_solve.argtypes = [ctypes.c_int] * 3 + [dp] * 5 + [ctypes.POINTER(Counter), ip, ip]
        L.or_dm_solve.argtypes = ([ctypes.c_int] * 4 + [ip, ctypes.c_int, ctypes.c_int] + [dp] * 5 +
                                  [ctypes.POINTER(_Aux), ctypes.POINTER(Counter), ctypes.c_int, ip, ip])
        L.or_gepp_solve.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.or_residual.argtypes = [ctypes.c_int] * 3 + [dp] * 6
        L.or_residual.restype = None
        L.or_max_threads.argtypes = []
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, row=-1, col=-1):
        super().__init__(f"oracle status {code} (block row {row}, column {col})")
        self.code, self.row, self.col = code, row, col


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check_shapes(A, B, C, F):
    N, M, M2 = A.shape
    assert M == M2 and B.shape == A.shape and C.shape == A.shape
    assert F.ndim == 3 and F.shape[:2] == (N, M)
    return N, M, F.shape[2]


def inverse(D):
    D = _f64(D)
    n = D.shape[0]
    G = np.empty_like(D)
    s = lib().or_inverse(n, _ptr(D), _ptr(G))
    if s:
        raise OracleError(1, -1, s - 1)
    return G


def partition(N, P):
    """Equal-split separator rows (0-based), length P-1."""
    seps = (ctypes.c_int * max(P - 1, 1))()
    s = lib().or_partition(N, P, seps)
    if s:
        raise ValueError(f"invalid partition N={N} P={P}")
    return [seps[i] for i in range(P - 1)]


def balanced_partition(N, P, alpha=7.0 / 4.0, beta=7.0 / 6.0):
    """Separator rows (0-based, length P-1) with subsystem sizes
    n_1 = alpha x, n_P = beta x and x for the others, x = (N - (P-1)) /
    (P - 2 + alpha + beta) (Sec. 5.1, second case, Eq. SpeedupMPNk).  Whole rows: the two end
    sizes rounded to the nearest row (at least one), shortened alternately
    (the longer first) while the middle subsystems would get less than one
    row each; the remaining rows split evenly over the middle subsystems,
    the leading ones one row longer."""
    if N < 1 or P < 1 or (P > 1 and 2 * P - 1 > N):
        raise ValueError(f"invalid partition N={N} P={P}")
    if P == 1:
        return []
    rows = N - (P - 1)
    x = rows / (P - 2 + alpha + beta)
    first = max(1, int(np.floor(alpha * x + 0.5)))
    last = max(1, int(np.floor(beta * x + 0.5)))
    if P == 2:
        first = min(first, rows - 1)
        sizes = [first, rows - first]
    else:
        while rows - first - last < P - 2:
            if first >= last:
                first -= 1
            else:
                last -= 1
        q, r = divmod(rows - first - last, P - 2)
        sizes = [first] + [q + (1 if k < r else 0) for k in range(P - 2)] + [last]
    seps, pos = [], 0
    for n in sizes[:-1]:
        pos += n
        seps.append(pos)
        pos += 1
    return seps


def default_m(P, M, R):
    return lib().or_default_m(P, M, R)


def ta_solve(A, B, C, F, counter=None):
    A, B, C, F = map(_f64, (A, B, C, F))
    N, M, R = _check_shapes(A, B, C, F)
    X = np.zeros_like(F)
    row, col = ctypes.c_int(-1), ctypes.c_int(-1)
    s = lib().or_ta_solve(N, M, R, _ptr(A), _ptr(B), _ptr(C), _ptr(F), _ptr(X),
                          ctypes.byref(counter) if counter is not None else None,
                          ctypes.byref(row), ctypes.byref(col))
    if s:
        raise OracleError(s, row.value, col.value)
    return X


def dm_solve(A, B, C, F, P, seps=None, depth=0, counter=None, want_aux=False, nthreads=0, J=1):
    """DM solve.  Returns X, or (X, aux dict) with want_aux.  J >= 2 solves
    every subsystem by the DM with J sub-subsystems (Sec. 4.2.2; D, E, y of
    aux are then not filled).

    aux holds D, E, ZL, ZR (shape (N, M, M), chunk rows only, zero elsewhere),
    y and z (shape (N, M, R)), Hd, Hb, Hc (shape (P-1, M, M)), fhat and h
    (shape (P-1, M, R)).
    """
    A, B, C, F = map(_f64, (A, B, C, F))
    N, M, R = _check_shapes(A, B, C, F)
    X = np.zeros_like(F)
    aux_np, aux_c = None, None
    if want_aux:
        Pc = max(P - 1, 0)
        aux_np = {k: np.zeros((N, M, M)) for k in ("D", "E", "ZL", "ZR")}
        aux_np.update({k: np.zeros((N, M, R)) for k in ("y", "z")})
        aux_np.update({k: np.zeros((Pc, M, M)) for k in ("Hd", "Hb", "Hc")})
        aux_np.update({k: np.zeros((Pc, M, R)) for k in ("fhat", "h")})
        aux_c = _Aux(**{k: (v.ctypes.data if v.size else None) for k, v in aux_np.items()})
    sep_arr = None
    if seps is not None:
        sep_arr = (ctypes.c_int * max(len(seps), 1))(*[int(s) for s in seps])
        assert len(seps) == P - 1
    row, col = ctypes.c_int(-1), ctypes.c_int(-1)
    s = lib().or_dm_solve(N, M, R, P, sep_arr, depth, int(J), _ptr(A), _ptr(B), _ptr(C), _ptr(F), _ptr(X),
                          ctypes.byref(aux_c) if aux_c is not None else None,
                          ctypes.byref(counter) if counter is not None else None,
                          int(nthreads), ctypes.byref(row), ctypes.byref(col))
    if s:
        raise OracleError(s, row.value, col.value)
    return (X, aux_np) if want_aux else X


def gepp_solve(Ad, Fd):
    """Dense GEPP solve of Ad (n x n) X = Fd (n x nrhs)."""
    Ad, Fd = _f64(Ad), _f64(Fd)
    if Fd.ndim == 1:
        Fd = Fd[:, None]
    n, nrhs = Fd.shape
    X = np.zeros_like(Fd)
    s = lib().or_gepp_solve(n, nrhs, _ptr(Ad), _ptr(Fd), _ptr(X))
    if s:
        raise OracleError(1, -1, s - 1)
    return X


def residual(A, B, C, X, F):
    """Per-column ||F - A X||_2 / ||F||_2 (numpy array of length R)."""
    A, B, C, X, F = map(_f64, (A, B, C, X, F))
    N, M, R = _check_shapes(A, B, C, F)
    out = np.zeros(R)
    lib().or_residual(N, M, R, _ptr(A), _ptr(B), _ptr(C), _ptr(X), _ptr(F), _ptr(out))
    return out


def dense(A, B, C):
    """Assemble the (N M) x (N M) dense matrix of the block-tridiagonal system
    (B_0 and C_{N-1} are not part of it)."""
    A, B, C = map(_f64, (A, B, C))
    N, M, _ = A.shape
    D = np.zeros((N * M, N * M))
    for i in range(N):
        D[i * M:(i + 1) * M, i * M:(i + 1) * M] = A[i]
        if i > 0:
            D[i * M:(i + 1) * M, (i - 1) * M:i * M] = B[i]
        if i < N - 1:
            D[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = C[i]
    return D


def max_threads():
    return lib().or_max_threads()
