"""Algorithmic FLOP counts of the decomposition method per kernel class.

Convention (LU form): LU of an M x M block with partial pivoting 2/3 M^3,
applying the factors to an M x r block 2 M^2 r, a product of an M x M block
with an M x r block 2 M^2 r.  These are the operations the method must do,
counted the way the paper counts block operations (Sec. 4, Tab. 1 and Tab. 2:
zero blocks of the spike right-hand sides are skipped), not the dense
(N M)^3 work it avoids and not any padding the kernels add.

The partition of every recursion level is taken from the library's own host
helpers, so the counts describe exactly the plan btd_factor builds.
"""
from . import btd

CLASSES = btd.KERNEL_CLASSES


def levels(N, M, P, depth, max_nrhs, seps=None, coupling_rows=0, sub_parts=0):
    """[(N_l, P_l, separators_l)] of every recursion level of a plan (the
    rule of btd_factor; with sub_parts J >= 2 the top level has P J
    subsystems and the next one splits at the P - 1 outer separators)."""
    out = []
    J = sub_parts if sub_parts >= 2 else 1
    if J > 1:
        outer = list(seps) if seps is not None else btd.default_separators(N, P)
        b = [-1] + outer + [N]
        s0 = []
        for k in range(P):
            r, nk = b[k] + 1, b[k + 1] - b[k] - 1
            s0 += [r + q for q in btd.default_separators(nk, J)]
            if k < P - 1:
                s0.append(b[k + 1])
        out.append((N, P * J, s0))
        N = P * J - 1
        s1 = [k * J + J - 1 for k in range(P - 1)]
        out.append((N, P, s1))
        if P == 1:
            return out
        Pc = btd.coupling_parts(P, M, max_nrhs, coupling_rows) if depth > 0 else 1
        N, P, depth = P - 1, Pc, max(depth - 1, 0)
        seps = None
    top = J == 1
    while True:
        s = list(seps) if (top and seps is not None) else btd.default_separators(N, P)
        out.append((N, P, s))
        if P == 1:
            return out
        Pc = btd.coupling_parts(P, M, max_nrhs, coupling_rows) if depth > 0 else 1
        N, P, depth, top = P - 1, Pc, max(depth - 1, 0), False


def chunk_sizes(N, P, seps):
    b = [-1] + list(seps) + [N]
    return [b[k + 1] - b[k] - 1 for k in range(P)]


def per_class(N, M, R, P, depth=0, max_nrhs=None, seps=None, coupling_rows=0, sub_parts=0):
    """Dict kernel class -> (total algorithmic FLOPs, number of launch steps).

    The launch-step count is that of one stream; when the plan splits a
    level's chunks into groups on several streams each step is that many
    launches.  diag_prep (inverses of the 32x32 diagonal blocks of the LU
    factors, used by the triangular solves) is a reformulation of the
    triangular solves, not an operation of the method: 0 algorithmic FLOPs."""
    max_nrhs = max_nrhs or R
    M3, M2R = float(M) ** 3, float(M) ** 2 * R
    tot = {c: 0.0 for c in CLASSES}
    launches = {c: 0 for c in CLASSES}
    for (Nl, Pl, s) in levels(N, M, P, depth, max_nrhs, seps, coupling_rows, sub_parts):
        nk = chunk_sizes(Nl, Pl, s)
        nmax = max(nk)
        for k, n in enumerate(nk):
            left, right = k > 0, k < Pl - 1
            tot["getrf"] += n * 2.0 / 3.0 * M3
            tot["fwd_gemm"] += (n - 1) * 2 * M3 * (1 + left)
            e_rows = n if right else n - 1
            tot["getrs_factor"] += 2 * M3 * (e_rows + (n if left else 0))
            if Pl > 1:
                tot["bwd_gemm"] += (n - 1) * 2 * M3 * (left + right)
                tot["recover"] += n * 2 * M2R * (left + right)
            # forward: (n-1) products with B, n applications of the LU factors; backward: (n-1) with E
            tot["rhs_sweep"] += ((n - 1) + n + (n - 1)) * 2 * M2R
        if Pl > 1:
            for j in range(Pl - 1):
                tot["couple"] += 2 * M3 * (2 + (j >= 1) + (j + 1 <= Pl - 2))
                tot["couple_rhs"] += 2 * 2 * M2R
        launches["fwd_gemm"] += nmax
        launches["getrf"] += nmax
        launches["getrs_factor"] += nmax
        launches["diag_prep"] += nmax
        launches["rhs_sweep"] += 1
        if Pl > 1:
            launches["bwd_gemm"] += nmax
            launches["couple"] += 1
            launches["couple_rhs"] += 1
            launches["recover"] += 1
    # residual: 3 block products per row (HBM-bound check, not part of the method)
    tot["residual"] = 2.0 * M * M * R * (3 * N - 2)
    launches["residual"] = 1
    return {c: (tot[c], launches[c]) for c in CLASSES}


FACTOR_CLASSES = ("fwd_gemm", "getrf", "getrs_factor", "bwd_gemm", "couple")
SOLVE_CLASSES = ("rhs_sweep", "couple_rhs", "recover")


def totals(N, M, R, P, depth=0, max_nrhs=None, seps=None, coupling_rows=0, sub_parts=0):
    """(factor FLOPs, solve FLOPs) of the method (residual excluded)."""
    pc = per_class(N, M, R, P, depth, max_nrhs, seps, coupling_rows, sub_parts)
    return sum(pc[c][0] for c in FACTOR_CLASSES), sum(pc[c][0] for c in SOLVE_CLASSES)


def unique_bytes(N, M, R):
    """Bytes the whole path must at least move once: read A, B, C, F and write X (FP64)."""
    return 8.0 * (3.0 * N * M * M + 2.0 * N * M * R)
