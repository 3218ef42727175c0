"""Many independent block-tridiagonal systems of uneven sizes solved together.

Systems with the same block size M are laid out one after another in one
block-tridiagonal system (A, B, C stacked along the rows) whose blocks
between two systems are zero: the B block of every system's first row and
the C block of its last row, which are not part of the system, are set to
zero.  That matrix is block diagonal over the systems, so one plan of the
library over it solves all of them; its subsystems may straddle the
junctions (a zero block only makes the elimination step there trivial), and
every kernel launch of a factor or solve step covers the subsystems of all
the systems of that block size at once.  Right-hand sides are stacked the
same way with the group's largest column count (columns a system does not
use are zero).

Plan parameters per group (rows per subsystem, how the coupling systems are
split) come from a small autotuner: candidates seeded by the paper's
optimum for the Thomas-algorithm cost model (Eq. MAXSpeedP for the rows per
subsystem, Eq. SuppMatrM or one-row coupling subsystems), each timed once on
the device, the fastest kept per (M, rows, columns, precision) key.

The arithmetic is the library's; this module stacks arrays (device copies)
and picks parameters.
"""
import ctypes
import math
import time

import numpy as np

from . import btd


def _torch():
    import torch
    return torch


class Group:
    """Systems of one block size M stacked into one system on the device."""

    def __init__(self, M, rows, nrhs, A, B, C, offsets):
        self.M = M
        self.rows = list(rows)            # N of every system
        self.nrhs = list(nrhs)            # R of every system
        self.A, self.B, self.C = A, B, C  # (sum N, M, M) device tensors, junction blocks zero
        self.offsets = list(offsets)      # first stacked row of every system
        self.N = int(sum(rows))
        self.R = int(max(nrhs))

    @staticmethod
    def stack(blocks, nrhs, device="cuda"):
        """blocks: list of (A, B, C) arrays of one M (numpy or torch, (N_s, M, M)).
        Copies them into stacked device arrays with the junction blocks zeroed."""
        torch = _torch()
        M = blocks[0][0].shape[1]
        rows = [a.shape[0] for a, _, _ in blocks]
        offsets = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(int)
        N = int(sum(rows))
        out = [torch.empty((N, M, M), dtype=torch.float64, device=device) for _ in range(3)]
        for (a, b, c), off, n in zip(blocks, offsets, rows):
            for dst, src in zip(out, (a, b, c)):
                src = torch.as_tensor(src)
                dst[off:off + n].copy_(src.to(device, non_blocking=False))
            out[1][off].zero_()           # B of the system's first row
            out[2][off + n - 1].zero_()   # C of its last row
        return Group(M, rows, nrhs, *out, offsets)

    def stack_rhs(self, Fs):
        """Per-system right-hand sides (N_s, M, R_s) into one (N, M, R) array."""
        torch = _torch()
        F = torch.zeros((self.N, self.M, self.R), dtype=torch.float64, device=self.A.device)
        for f, off, n, r in zip(Fs, self.offsets, self.rows, self.nrhs):
            F[off:off + n, :, :r].copy_(torch.as_tensor(f).to(self.A.device))
        return F

    def split(self, X):
        """The stacked solution back into per-system (N_s, M, R_s) views."""
        return [X[off:off + n, :, :r] for off, n, r in zip(self.offsets, self.rows, self.nrhs)]


def max_speed_p(N, n, l):
    """Eq. MAXSpeedP: the subsystem count of the largest speedup of Eq.
    SpeedupMP for N block rows, block size n and l right-hand sides."""
    return math.sqrt((N + 1) / 3.0 * (5.0 + 2.0 / (1.0 + l / n)))


class Tuner:
    """Rows per subsystem and coupling split for a stacked group, chosen by
    timing a few candidates once and cached.

    Candidates: the mean system's rows over Eq. MAXSpeedP's subsystem count
    (the paper's optimum for one processor per subsystem), and 8, 16 and 32
    rows (on the GPU every subsystem of a step runs in the same launch, so
    shorter subsystems mean fewer sequential steps); each with one-row
    coupling subsystems (depth 10) and with Eq. SuppMatrM's split (depth 2).
    fused: candidates timed as one btd_factor_solve call (prec f64)."""

    def __init__(self, fused=False):
        self.fused = fused
        self.cache = {}
        self.log = []

    def key(self, g, prec):
        return (g.M, int(round(math.log2(max(g.N, 1)))), g.R, prec)

    def candidates(self, g):
        mean_rows = g.N / len(g.rows)
        p_star = max_speed_p(mean_rows, g.M, g.R)
        seeded = max(2, int(round(mean_rows / p_star)))
        rows = sorted({seeded, 8, 16, 32})
        return [(r, 10, 1) for r in rows] + [(r, 2, 0) for r in rows[:2]]

    @staticmethod
    def parts(g, rows):
        """Subsystem count for about `rows` rows per subsystem (at least one row each)."""
        return max(1, min((g.N + 1) // (rows + 1), (g.N + 1) // 2))

    def choose(self, g, F, prec="f64"):
        k = self.key(g, prec)
        if k in self.cache:
            return self.cache[k]
        torch = _torch()
        best = None
        for rows, depth, crow in self.candidates(g):
            P = self.parts(g, rows)
            run = GroupRun(g, P, depth, crow, prec, fused=self.fused)
            run.step(F)            # warm (also builds the workspaces)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.step(F)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            run.release()
            del run
            torch.cuda.empty_cache()
            self.log.append({"M": g.M, "N": g.N, "R": g.R, "rows": rows, "P": P, "depth": depth,
                             "coupling_rows": crow, "ms": ms})
            if best is None or ms < best[0]:
                best = (ms, P, depth, crow)
        self.cache[k] = best[1:]
        return self.cache[k]


class GroupRun:
    """Factor + solve of one stacked group through the C ABI with workspaces
    allocated once (graph-capturable for prec f64)."""

    def __init__(self, g, P, depth, coupling_rows, prec="f64", stream=None, shared=None, fused=False):
        """shared: optional (factor buffer, solve buffer) uint8 tensors at least
        as large as this plan needs, reused by groups run one after another on
        one stream.  fused (prec f64): factor and solve in one
        btd_factor_solve call."""
        torch = _torch()
        self.g, self.prec = g, prec
        self.fused = fused and prec == "f64"
        self.P, self.depth, self.coupling_rows = P, depth, coupling_rows
        self.L = btd.lib()
        self.desc, self._keep = btd.make_desc(g.N, g.M, P, depth, g.R, None, coupling_rows, prec)
        self.fb, self.sb = btd.workspace_bytes(g.N, g.M, P, depth, g.R, None, coupling_rows)
        if shared is None:
            self.fws, self.fptr = btd._aligned_buffer(self.fb, g.A.device)
            self.sws, self.sptr = btd._aligned_buffer(self.sb, g.A.device)
        else:
            self.fws, self.sws = shared
            self.fptr = (self.fws.data_ptr() + 255) // 256 * 256
            self.sptr = (self.sws.data_ptr() + 255) // 256 * 256
            assert self.fptr + self.fb <= self.fws.data_ptr() + self.fws.numel()
            assert self.sptr + self.sb <= self.sws.data_ptr() + self.sws.numel()
        self.X = torch.zeros((g.N, g.M, g.R), dtype=torch.float64, device=g.A.device)
        self.plans = []
        self.rws = None
        self.iters, self.res = [], []
        self.use_stream(stream or torch.cuda.current_stream(g.A.device))

    def use_stream(self, s):
        self.stream = s
        self.sh = ctypes.c_void_p(s.cuda_stream)

    def step(self, F):
        """Factor and solve (refined to 1e-12 for prec f32_refine, which
        blocks on the residual norms)."""
        g, L = self.g, self.L
        h = ctypes.c_void_p()
        if self.fused:
            rc = L.btd_factor_solve(ctypes.byref(self.desc), g.A.data_ptr(), g.B.data_ptr(), g.C.data_ptr(),
                                    self.fptr, self.fb, g.R, F.data_ptr(), self.X.data_ptr(), self.sptr, self.sb,
                                    self.sh, ctypes.byref(h))
            if rc:
                raise btd.BtdError(rc, "btd_factor_solve")
            self.plans.append(h)
            return self.X
        rc = L.btd_factor(ctypes.byref(self.desc), g.A.data_ptr(), g.B.data_ptr(), g.C.data_ptr(), self.fptr,
                          self.fb, self.sh, ctypes.byref(h))
        if rc:
            raise btd.BtdError(rc, "btd_factor")
        self.plans.append(h)
        if self.prec == "f32_refine":
            if self.rws is None:
                nb = L.btd_refine_work_bytes(h, g.R)
                self.rws, self.rptr = btd._aligned_buffer(nb, g.A.device)
                self.rb = nb
            it, res = ctypes.c_int32(), ctypes.c_double()
            rc = L.btd_solve_refine(h, g.R, F.data_ptr(), self.X.data_ptr(), self.rptr, self.rb, ctypes.c_double(1e-12),
                                    8, ctypes.byref(it), ctypes.byref(res), self.sh)
            if rc:
                raise btd.BtdError(rc, f"btd_solve_refine (residual {res.value:.2e})")
            self.iters.append(it.value)
            self.res.append(res.value)
        else:
            rc = L.btd_solve(h, g.R, F.data_ptr(), self.X.data_ptr(), self.sptr, self.sb, self.sh)
            if rc:
                raise btd.BtdError(rc, "btd_solve")
        return self.X

    def info(self):
        st, row, col = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _torch().cuda.synchronize()
        self.L.btd_get_info(self.plans[-1], ctypes.byref(st), ctypes.byref(row), ctypes.byref(col))
        return st.value, row.value, col.value

    def release(self):
        _torch().cuda.synchronize()
        for h in self.plans:
            self.L.btd_plan_destroy(h)
        self.plans = []


def group_by_block_size(specs):
    """specs: list of (N, M, R) per system -> {M: [system indices]} (order kept)."""
    groups = {}
    for s, (N, M, R) in enumerate(specs):
        groups.setdefault(M, []).append(s)
    return groups
