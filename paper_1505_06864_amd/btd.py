"""Python binding of libbtd.so (include/btd.h): argument marshalling only.

Every step of the factor and the solve runs in the library's HIP kernels;
this module converts torch tensors to device pointers, allocates the
workspaces the C ABI asks for (torch owns all device memory), and passes the
current HIP stream.  There is no CPU fallback: without the built library on
a HIP device the calls raise.

Shapes (row-major, torch.float64 on a HIP device): A, B, C (N, M, M) --
diagonal, sub-diagonal, super-diagonal blocks of
B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i; F, X (N, M, R).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbtd.so")

BTD_OK, BTD_ERR_SINGULAR, BTD_ERR_NONFINITE, BTD_ERR_LAUNCH, BTD_ERR_SCRATCH, BTD_ERR_NOT_CONVERGED = 0, 1, 2, 3, 4, 5
NOALLOC_SCRATCH_BYTES = 64 << 20
BTD_PREC_F64 = 0
BTD_PREC_F32_REFINE = 1
PRECISIONS = {"f64": BTD_PREC_F64, "f32_refine": BTD_PREC_F32_REFINE}
BTD_MAX_M = 512

# Every symbol include/btd.h declares.
EXPORTS = ("btd_workspace_bytes", "btd_factor", "btd_factor_solve", "btd_solve", "btd_solve_batch", "btd_solve_noalloc", "btd_refine_work_bytes", "btd_solve_refine", "btd_solve_local",
           "btd_solve_finish", "btd_get_solve_info", "btd_plan_level_arrays", "btd_residual_work_bytes",
           "btd_residual", "btd_get_info", "btd_plan_separators", "btd_plan_level_parts",
           "btd_default_separators", "btd_balanced_separators", "btd_default_coupling_parts",
           "btd_coupling_parts", "btd_profile_enable", "btd_profile_read",
           "btd_plan_destroy", "btd_status_string")

# Kernel classes of btd_profile_enable (BTD_KC_*).
KERNEL_CLASSES = ("fwd_gemm", "getrf", "getrs_factor", "bwd_gemm", "couple", "rhs_sweep", "couple_rhs",
                  "recover", "residual", "diag_prep")


class Desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("P", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("prec", ctypes.c_int32), ("max_nrhs", ctypes.c_int32),
                ("seps", ctypes.POINTER(ctypes.c_int32)), ("coupling_rows", ctypes.c_int32),
                ("sub_parts", ctypes.c_int32)]


class LevelArrays(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("P", ctypes.c_int32)] + \
               [(n, ctypes.c_void_p) for n in ("A", "B", "C", "W", "Z", "Hd", "Hb", "Hc", "sep")]


_lib = None


def lib():
    """Load libbtd.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1505_06864_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        L.btd_workspace_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.btd_factor.argtypes = [ctypes.POINTER(Desc), vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
        L.btd_factor_solve.argtypes = [ctypes.POINTER(Desc), vp, vp, vp, vp, sz, i32, vp, vp, vp, sz, vp,
                                       ctypes.POINTER(vp)]
        L.btd_solve.argtypes = [vp, i32, vp, vp, vp, sz, vp]
        L.btd_solve_batch.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), vp, sz, vp]
        L.btd_solve_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.btd_refine_work_bytes.argtypes = [vp, i32]
        L.btd_refine_work_bytes.restype = sz
        L.btd_solve_refine.argtypes = [vp, i32, vp, vp, vp, sz, ctypes.c_double, i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(ctypes.c_double), vp]
        L.btd_solve_local.argtypes = [vp, i32, vp, vp, vp, vp]
        L.btd_solve_finish.argtypes = [vp, i32, vp, vp, vp]
        L.btd_get_solve_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.btd_plan_level_arrays.argtypes = [vp, i32, ctypes.POINTER(LevelArrays)]
        L.btd_residual_work_bytes.argtypes = [i32, i32, i32]
        L.btd_residual_work_bytes.restype = sz
        L.btd_residual.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.btd_get_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.btd_plan_separators.argtypes = [vp, ctypes.POINTER(i32)]
        L.btd_plan_level_parts.argtypes = [vp, i32]
        L.btd_default_separators.argtypes = [i32, i32, ctypes.POINTER(i32)]
        L.btd_balanced_separators.argtypes = [i32, i32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(i32)]
        L.btd_default_coupling_parts.argtypes = [i32, i32, i32]
        L.btd_coupling_parts.argtypes = [i32, i32, i32, i32]
        L.btd_profile_enable.argtypes = [i32]
        L.btd_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.btd_plan_destroy.argtypes = [vp]
        L.btd_plan_destroy.restype = None
        L.btd_status_string.argtypes = [ctypes.c_int]
        L.btd_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


class BtdError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().btd_status_string(code).decode()
        super().__init__(f"{what}: code {code} ({msg})")
        self.code = code


def _torch():
    import torch
    return torch


def _check(t, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch.float64 tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _stream_handle(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _empty_on(stream, *args, **kw):
    """torch.empty allocated on `stream` (None = the current stream): the
    caching allocator then reuses the memory only in that stream's order, so
    a buffer the library's kernels use on `stream` is never handed to other
    work while they may still run."""
    torch = _torch()
    if stream is None:
        return torch.empty(*args, **kw)
    with torch.cuda.stream(stream):
        return torch.empty(*args, **kw)


def _aligned_buffer(nbytes, device, stream=None):
    """A torch uint8 buffer (allocated on `stream`) and a 256-byte-aligned pointer inside it."""
    torch = _torch()
    buf = _empty_on(stream, nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (buf.data_ptr() + 255) // 256 * 256
    return buf, ptr


def make_desc(N, M, P=1, depth=0, max_nrhs=1, seps=None, coupling_rows=0, prec="f64", sub_parts=0):
    d = Desc(N, M, P, depth, PRECISIONS[prec], max_nrhs, None, coupling_rows, sub_parts)
    keep = None
    if seps is not None:
        keep = (ctypes.c_int32 * max(len(seps), 1))(*[int(q) for q in seps])
        d.seps = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
    return d, keep


def workspace_bytes(N, M, P=1, depth=0, max_nrhs=1, seps=None, coupling_rows=0, sub_parts=0):
    """(factor bytes, solve bytes) for a description; raises on an invalid one."""
    d, _keep = make_desc(N, M, P, depth, max_nrhs, seps, coupling_rows, sub_parts=sub_parts)
    f, s = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib().btd_workspace_bytes(ctypes.byref(d), ctypes.byref(f), ctypes.byref(s))
    if rc != BTD_OK:
        raise BtdError(rc, "btd_workspace_bytes")
    return f.value, s.value


def default_separators(N, P):
    """Equal-split separator rows the library uses when none are given (host only)."""
    out = (ctypes.c_int32 * max(P - 1, 1))()
    rc = lib().btd_default_separators(N, P, out)
    if rc != BTD_OK:
        raise BtdError(rc, "btd_default_separators")
    return [out[k] for k in range(P - 1)]


def balanced_separators(N, P, alpha=7.0 / 4.0, beta=7.0 / 6.0):
    """Separator rows of the balanced partition (Sec. 5.1, Eq. SpeedupMPNk: first and last
    subsystems alpha and beta times the middle ones), host only."""
    out = (ctypes.c_int32 * max(P - 1, 1))()
    rc = lib().btd_balanced_separators(N, P, ctypes.c_double(alpha), ctypes.c_double(beta), out)
    if rc != BTD_OK:
        raise BtdError(rc, "btd_balanced_separators")
    return [out[k] for k in range(P - 1)]


def default_coupling_parts(P, M, R):
    """Subsystem count of the recursive coupling solve, Eq. SuppMatrM (host only)."""
    rc = lib().btd_default_coupling_parts(P, M, R)
    if rc < 0:
        raise BtdError(rc, "btd_default_coupling_parts")
    return rc


def coupling_parts(P, M, R, coupling_rows=0):
    """Subsystem count of the coupling solve for a coupling_rows setting (host only)."""
    rc = lib().btd_coupling_parts(P, M, R, coupling_rows)
    if rc < 0:
        raise BtdError(rc, "btd_coupling_parts")
    return rc


class Plan:
    """A factored system (btd_factor).  Keeps A, B, C and the factor workspace alive.

    With F given the plan is built by btd_factor_solve, which also solves
    for F in the same call (into X, or a new array); the solution is
    ``self.X``."""

    def __init__(self, A, B, C, P=1, depth=0, max_nrhs=1, seps=None, stream=None, coupling_rows=0, prec="f64",
                 sub_parts=0, F=None, X=None):
        N, M = A.shape[0], A.shape[1]
        for t, n in ((A, "A"), (B, "B"), (C, "C")):
            _check(t, n, (N, M, M))
        self.N, self.M, self.P, self.depth, self.max_nrhs, self.prec = N, M, P, depth, max_nrhs, prec
        self.device = A.device
        self.A, self.B, self.C = A, B, C
        fbytes, self.solve_bytes = workspace_bytes(N, M, P, depth, max_nrhs, seps, coupling_rows, sub_parts)
        self._ws, ptr = _aligned_buffer(fbytes, A.device, stream)
        d, _keep = make_desc(N, M, P, depth, max_nrhs, seps, coupling_rows, prec, sub_parts)
        h = ctypes.c_void_p()
        self.X = None
        if F is None:
            rc = lib().btd_factor(ctypes.byref(d), A.data_ptr(), B.data_ptr(), C.data_ptr(), ptr, fbytes,
                                  _stream_handle(stream, A.device), ctypes.byref(h))
            if rc != BTD_OK:
                raise BtdError(rc, "btd_factor")
        else:
            R = F.shape[2]
            _check(F, "F", (N, M, R))
            if X is None:
                X = _empty_on(stream, F.shape, dtype=F.dtype, device=F.device)
            _check(X, "X", (N, M, R))
            buf, sptr = _aligned_buffer(self.solve_bytes, F.device, stream)
            rc = lib().btd_factor_solve(ctypes.byref(d), A.data_ptr(), B.data_ptr(), C.data_ptr(), ptr, fbytes, R,
                                        F.data_ptr(), X.data_ptr(), sptr, self.solve_bytes,
                                        _stream_handle(stream, A.device), ctypes.byref(h))
            if rc != BTD_OK:
                raise BtdError(rc, "btd_factor_solve")
            self._last_solve_ws = buf
            self.X = X
        self._h = h
        self.factor_bytes = fbytes

    @property
    def handle(self):
        return self._h

    def solve(self, F, X=None, stream=None):
        """X = A^{-1} F (X may be F for an in-place solve).  Returns X."""
        R = F.shape[2]
        _check(F, "F", (self.N, self.M, R))
        if X is None:
            X = _empty_on(stream, F.shape, dtype=F.dtype, device=F.device)
        _check(X, "X", (self.N, self.M, R))
        buf, ptr = _aligned_buffer(self.solve_bytes, F.device, stream)
        rc = lib().btd_solve(self._h, R, F.data_ptr(), X.data_ptr(), ptr, self.solve_bytes,
                             _stream_handle(stream, F.device))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_solve")
        self._last_solve_ws = buf  # lives until the next solve on this plan (stream-ordered reuse)
        return X

    def solve_refine(self, F, X=None, tol=1e-12, max_iter=5, stream=None):
        """Iteratively refined solve (btd_solve_refine; blocking).  Returns
        (X, corrections made, final max relative residual); raises
        BtdError(BTD_ERR_NOT_CONVERGED) when tol is not reached."""
        R = F.shape[2]
        _check(F, "F", (self.N, self.M, R))
        if X is None:
            X = _empty_on(stream, F.shape, dtype=F.dtype, device=F.device)
        _check(X, "X", (self.N, self.M, R))
        nbytes = lib().btd_refine_work_bytes(self._h, R)
        buf, ptr = _aligned_buffer(nbytes, F.device, stream)
        it, res = ctypes.c_int32(), ctypes.c_double()
        rc = lib().btd_solve_refine(self._h, R, F.data_ptr(), X.data_ptr(), ptr, nbytes, ctypes.c_double(tol),
                                    max_iter, ctypes.byref(it), ctypes.byref(res), _stream_handle(stream, F.device))
        del buf   # the call synchronised its stream
        if rc != BTD_OK:
            raise BtdError(rc, f"btd_solve_refine (residual {res.value:.3e} after {it.value} corrections)")
        return X, it.value, res.value

    def solve_local(self, F, X=None, Fhat=None, stream=None):
        """The per-subsystem half of a solve (btd_solve_local): z into the
        subsystem rows of X and the coupling right-hand side into Fhat
        ((P-1, M, R)).  Returns (X, Fhat)."""
        torch = _torch()
        R = F.shape[2]
        _check(F, "F", (self.N, self.M, R))
        if X is None:
            X = _empty_on(stream, F.shape, dtype=F.dtype, device=F.device)
        _check(X, "X", (self.N, self.M, R))
        P0 = self.level_parts()[0]       # subsystems of the top level (P * sub_parts)
        if Fhat is None and P0 > 1:
            Fhat = _empty_on(stream, (P0 - 1, self.M, R), dtype=torch.float64, device=F.device)
        if Fhat is not None:
            _check(Fhat, "Fhat", (P0 - 1, self.M, R))
        rc = lib().btd_solve_local(self._h, R, F.data_ptr(), X.data_ptr(),
                                   Fhat.data_ptr() if Fhat is not None else None, _stream_handle(stream, F.device))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_solve_local")
        return X, Fhat

    def solve_finish(self, H, X, stream=None):
        """Recovery from the coupling solution H ((P-1, M, R)) into X (btd_solve_finish)."""
        R = X.shape[2]
        _check(X, "X", (self.N, self.M, R))
        P0 = self.level_parts()[0]
        if P0 > 1:
            _check(H, "H", (P0 - 1, self.M, R))
        rc = lib().btd_solve_finish(self._h, R, H.data_ptr() if H is not None else None, X.data_ptr(),
                                    _stream_handle(stream, X.device))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_solve_finish")
        return X

    def level_arrays(self, level=0):
        """Read-only device views of one recursion level (btd_plan_level_arrays)
        as torch tensors sharing the workspace memory: dict with N, M, P and
        W (N, M, 2M), Z (N, M, 2M) and Hd, Hb, Hc (P-1, M, M) (None when P = 1)
        and sep (P+1,)."""
        torch = _torch()
        out = LevelArrays()
        rc = lib().btd_plan_level_arrays(self._h, level, ctypes.byref(out))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_plan_level_arrays")
        N, M, P = out.N, out.M, out.P
        base = self._ws.data_ptr()
        u8 = self._ws

        def view(ptr, shape, dtype=torch.float64, esize=8):
            if not ptr:
                return None
            n = 1
            for d in shape:
                n *= d
            off = ptr - base
            assert 0 <= off and off + n * esize <= u8.numel(), "view outside the factor workspace"
            return u8[off:off + n * esize].view(dtype).view(*shape)

        return {"N": N, "M": M, "P": P,
                "W": view(out.W, (N, M, 2 * M)), "Z": view(out.Z, (N, M, 2 * M)),
                "Hd": view(out.Hd, (P - 1, M, M)), "Hb": view(out.Hb, (P - 1, M, M)),
                "Hc": view(out.Hc, (P - 1, M, M)), "sep": view(out.sep, (P + 1,), torch.int32, 4)}

    def solve_info(self):
        """(status, block_row, col) of the right-hand-side check of the last
        solve; synchronises the device first."""
        _torch().cuda.synchronize(self.device)
        st, row, col = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rc = lib().btd_get_solve_info(self._h, ctypes.byref(st), ctypes.byref(row), ctypes.byref(col))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_get_solve_info")
        return st.value, row.value, col.value

    def info(self):
        """(status, block_row, col) of the factor; synchronises the device first."""
        _torch().cuda.synchronize(self.device)
        st, row, col = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rc = lib().btd_get_info(self._h, ctypes.byref(st), ctypes.byref(row), ctypes.byref(col))
        if rc != BTD_OK:
            raise BtdError(rc, "btd_get_info")
        return st.value, row.value, col.value

    def separators(self):
        out = (ctypes.c_int32 * max(self.P - 1, 1))()
        lib().btd_plan_separators(self._h, out)
        return [out[k] for k in range(self.P - 1)]

    def level_parts(self):
        parts, lvl = [], 0
        while True:
            p = lib().btd_plan_level_parts(self._h, lvl)
            if p < 0:
                return parts
            parts.append(p)
            lvl += 1

    def release_after_work(self):
        """Destroy the plan without waiting for the device: only for a plan
        whose enqueued work is known to have finished (its workspace returns
        to the stream it was allocated on)."""
        if getattr(self, "_h", None):
            lib().btd_plan_destroy(self._h)
            self._h = None
            self._ws = None
            self._last_solve_ws = None

    def destroy(self):
        if getattr(self, "_h", None):
            _torch().cuda.synchronize(self.device)
            lib().btd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def factor(A, B, C, P=1, depth=0, max_nrhs=1, seps=None, stream=None, coupling_rows=0, prec="f64", sub_parts=0):
    return Plan(A, B, C, P=P, depth=depth, max_nrhs=max_nrhs, seps=seps, stream=stream, coupling_rows=coupling_rows,
                prec=prec, sub_parts=sub_parts)


def factor_solve(A, B, C, F, X=None, P=1, depth=0, max_nrhs=None, seps=None, stream=None, coupling_rows=0,
                 prec="f64", sub_parts=0):
    """btd_factor_solve: factor and solve for F in one call.  Returns (plan, X)."""
    p = Plan(A, B, C, P=P, depth=depth, max_nrhs=max_nrhs or F.shape[2], seps=seps, stream=stream,
             coupling_rows=coupling_rows, prec=prec, sub_parts=sub_parts, F=F, X=X)
    return p, p.X


def solve_batch(plans, Fs, Xs=None, stream=None, lanes=1):
    """btd_solve_batch over several plans; returns the list of solutions.
    lanes > 1 gives the call room for that many solves side by side."""
    torch = _torch()
    n = len(plans)
    if Xs is None:
        Xs = [_empty_on(stream, F.shape, dtype=F.dtype, device=F.device) for F in Fs]
    nbytes = max(lanes, 1) * ((max(p.solve_bytes for p in plans) + 255) // 256 * 256) if n else 256
    buf, ptr = _aligned_buffer(nbytes, Fs[0].device if n else "cuda", stream)
    hp = (ctypes.c_void_p * max(n, 1))(*[p.handle.value for p in plans])
    nr = (ctypes.c_int32 * max(n, 1))(*[F.shape[2] for F in Fs])
    fp = (ctypes.c_void_p * max(n, 1))(*[F.data_ptr() for F in Fs])
    xp = (ctypes.c_void_p * max(n, 1))(*[X.data_ptr() for X in Xs])
    rc = lib().btd_solve_batch(n, hp, nr, fp, xp, ptr, nbytes,
                               _stream_handle(stream, Fs[0].device if n else None))
    if rc != BTD_OK:
        raise BtdError(rc, "btd_solve_batch")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    del buf
    return Xs


def profile_enable(kernel_class):
    """Bracket every launch of one kernel class (name or BTD_KC_* index, None = off) with HIP events."""
    idx = -1 if kernel_class is None else (KERNEL_CLASSES.index(kernel_class)
                                           if isinstance(kernel_class, str) else int(kernel_class))
    if lib().btd_profile_enable(idx) != BTD_OK:
        raise ValueError(f"unknown kernel class {kernel_class}")


def profile_read():
    """(total milliseconds, launches) of the enabled class since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    rc = lib().btd_profile_read(ctypes.byref(ms), ctypes.byref(n))
    if rc != BTD_OK:
        raise BtdError(rc, "btd_profile_read")
    return ms.value, n.value


def residual(A, B, C, X, F, stream=None):
    """Per-column ||F - A X||_2 / ||F||_2 computed on the device (tensor of R float64)."""
    torch = _torch()
    N, M, R = F.shape
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _check(t, nm, (N, M, M))
    _check(X, "X", (N, M, R))
    _check(F, "F", (N, M, R))
    out = _empty_on(stream, R, dtype=torch.float64, device=F.device)
    work = _empty_on(stream, max(lib().btd_residual_work_bytes(N, M, R), 8) // 8, dtype=torch.float64,
                     device=F.device)
    rc = lib().btd_residual(N, M, R, A.data_ptr(), B.data_ptr(), C.data_ptr(), X.data_ptr(), F.data_ptr(),
                            out.data_ptr(), work.data_ptr(), _stream_handle(stream, F.device))
    if rc != BTD_OK:
        raise BtdError(rc, "btd_residual")
    return out
