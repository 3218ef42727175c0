"""Closed-form cost model of the DM (arXiv:1505.06864, Sec. 4 and Sec. 5).

TEST INFRASTRUCTURE ONLY (part of the oracle).  Paper notation here:
n = block size, l = RHS columns, N = block rows, Nk = rows of subsystem k,
M = number of subsystems (the build calls it P), m = subsystems of the
coupling system, J = sub-subsystems per subsystem.  Costs are counts of
multiplicative operations in units of n^3 and n^2 l, returned as pairs
(a, b) meaning a n^3 + b n^2 l.
"""
import math

import numpy as np


def ta_table1(N):
    """Tab. 1: per-part counts of the Thomas algorithm and the total (3N-2)(n^3+n^2 l)."""
    parts = {"G": (2 * N - 1, 0), "script_A": (N - 1, 0), "script_B": (0, 2 * N - 1), "X": (0, N - 1)}
    total = (3 * N - 2, 3 * N - 2)
    assert tuple(map(sum, zip(*parts.values()))) == total
    return parts, total


def dm_table2_subsystem(k, P, Nk):
    """Tab. 2, 'solution of Eq. e231' row for subsystem k (1-based) of P."""
    if k == 1:
        return (4 * Nk - 2, 3 * Nk - 2)
    if k == P:
        return (6 * Nk - 4, 3 * Nk - 2)
    return (7 * Nk - 4, 3 * Nk - 2)


def dm_table2_coupling_products(k, P):
    """Tab. 2, products W_L^k Z^k and W_L^k z^k (Eq. e2311)."""
    return (1, 1) if k in (1, P) else (4, 2)


def dm_table2_recovery(k, P, Nk):
    """Tab. 2, products of Eq. endSolution."""
    return (0, Nk) if k in (1, P) else (0, 2 * Nk)


def dm_total(Nks, coupling=None):
    """Eq. DMtotal for subsystem sizes Nks (length P >= 2); the last term
    (3P-5)(n^3+n^2 l) is the TA on the coupling system unless `coupling`
    (a pair) replaces it (Eq. DMrec1)."""
    P = len(Nks)
    a = (4 * Nks[0] - 1) + (6 * Nks[-1] - 3) + sum(7 * x for x in Nks[1:-1])
    b = (4 * Nks[0] - 1) + (4 * Nks[-1] - 1) + sum(5 * x for x in Nks[1:-1])
    c = coupling if coupling is not None else (3 * P - 5, 3 * P - 5)
    return (a + c[0], b + c[1])


def dm_rec1(Nks, Mjs):
    """Eq. DMrec1: DMtotal with the coupling system (P-1 rows) split into
    subsystems of sizes Mjs and solved by the non-recursive DM."""
    return dm_total(Nks, coupling=dm_total(Mjs))


def speedup_mp(N, P, n, l):
    """Eq. SpeedupMP (equal subsystems, P = number of subsystems = processors)."""
    return (3 * N - 2) / (3 * P - 5 + (5 + 2 / (1 + l / n)) * ((N - P + 1) / P))


def speedup_mp_lower(N, P):
    """The lower bound printed with Eq. SpeedupMP."""
    return 1.0 / (7.0 / (3 * P) + P / N)


def speedup_optimal_P(N, n, l):
    """Maximiser of Eq. SpeedupMP over P (Eq. MAXSpeedP)."""
    return math.sqrt((N + 1) / 3 * (5 + 2 / (1 + l / n)))


def suppmatr_m(P, n, l):
    """Eq. SuppMatrM: optimal subsystem count of the coupling system."""
    return math.sqrt(P / 3 * (5 + 2 / (1 + l / n)))


def p3dmrec4(N, n, l):
    """Both recursions, P free: J from the cubic Eq. P3DMrec4, then M and m
    from Eq. P2DMrec4.  Returns (M, J, m) as floats."""
    a3 = 11 * n**3 + 5 * n**2 * l
    a7 = 7 * n**3 + 3 * n**2 * l
    two = 2 * n**2 * l
    c1 = a3 / two
    c0 = -(math.sqrt(N + 1) / two) * (a3 / a7) ** 1.5 * math.sqrt(
        3 * (7 * n**3 + 5 * n**2 * l) * (n**3 + n**2 * l))
    roots = np.roots([1.0, c1, 0.0, c0])
    J = max(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 0)
    M = (N + 1) / J**2 * (a3 / a7)
    m = math.sqrt(M * (7 * n**3 + 5 * n**2 * l) / (3 * (n**3 + n**2 * l)))
    return M, J, m


def dm_rec12(Ls, k, P):
    """Solution of Eq. e231 for subsystem k (1-based) of P by the DM with
    sub-subsystem sizes Ls (recursion into the subsystems, Sec. 4.2.2):
    Eq. DMrec121 (k = 1), Eq. DMrec1212 (k = P), Eq. DMrec122 (otherwise)."""
    J = len(Ls)
    L1, LJ, mid = Ls[0], Ls[-1], sum(Ls[1:-1])
    if k == 1:
        return ((5 * L1 - 1) + (8 * LJ - 2) + 9 * mid + (4 * J - 6),
                (4 * L1 - 1) + (4 * LJ - 1) + 5 * mid + (3 * J - 5))
    if k == P:
        return ((8 * L1 - 2) + (7 * LJ - 3) + 9 * mid + (6 * J - 10),
                (4 * L1 - 1) + (4 * LJ - 1) + 5 * mid + (3 * J - 5))
    return ((9 * L1 - 2) + (9 * LJ - 2) + 11 * mid + (7 * J - 11),
            (4 * L1 - 1) + (4 * LJ - 1) + 5 * mid + (3 * J - 5))


def dm_total_subrec(Ls_per_subsystem, coupling=None):
    """Total operations of the DM whose subsystems are solved by the DM
    (sizes Ls_per_subsystem[k] of their sub-subsystems): Eqs. DMrec121-122
    summed over the subsystems, plus the coupling products and the recovery
    of Tab. 2 and the coupling system ((3P-5)(n^3+n^2 l), or `coupling`)."""
    P = len(Ls_per_subsystem)
    parts = [dm_rec12(Ls, k, P) for k, Ls in enumerate(Ls_per_subsystem, 1)]
    Nks = [sum(Ls) + len(Ls) - 1 for Ls in Ls_per_subsystem]
    parts += [dm_table2_coupling_products(k, P) for k in range(1, P + 1)]
    parts += [dm_table2_recovery(k, P, Nk) for k, Nk in enumerate(Nks, 1)]
    parts.append(coupling if coupling is not None else (3 * P - 5, 3 * P - 5))
    return tuple(map(sum, zip(*parts)))


def dmrec3(N, M, J, n, l):
    """Eq. DMrec3: serial operations with M equal subsystems of J equal
    sub-subsystems each (P = M J processors), the coupling system by the
    Thomas algorithm."""
    N1 = (N - M + 1) / M
    N2 = (N1 - J + 1) / J
    return ((11 * n**3 + 5 * n**2 * l) * N2 + (n**3 * (7 * J - 11) + n**2 * l * (3 * J - 5))
            + 4 * n**3 + 2 * n**2 * l + (n**3 + n**2 * l) * (3 * M - 5) + 2 * n**2 * l * N1)


def p3dmrec3(N, n, l):
    """Recursion into the subsystems with P free: J the real positive root of
    the quartic Eq. P3DMrec3, M from Eq. P2DMrec3.  Returns (M, J)."""
    a11 = 11 * n**3 + 5 * n**2 * l
    a7 = 7 * n**3 + 3 * n**2 * l
    two = 2 * n**2 * l
    c3 = a11 / two
    c0 = -(N + 1) * 3 * (n**3 + n**2 * l) * a11**2 / (a7**2 * two)
    roots = np.roots([1.0, c3, 0.0, 0.0, c0])
    J = max(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 0)
    return (N + 1) / J**2 * (a11 / a7), J
