"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a library
routine (LAPACK through numpy), a closed form, a printed value of the paper,
an invariant, or brute force over tiny inputs.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import costmodel
from paper_1505_06864_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_system(N, M, R, seed, shift=2.0):
    return inputs.diag_dominant(N, M, R, seed, shift=shift)


def dense_solve(A, B, C, F):
    N, M, R = F.shape
    D = oracle.dense(A, B, C)
    return np.linalg.solve(D, F.reshape(N * M, R)).reshape(N, M, R)


def all_separator_sets(N, P):
    """Every choice of P-1 separators in rows 1..N-2 with non-empty subsystems."""
    for seps in itertools.combinations(range(1, N - 1), P - 1):
        if all(b - a >= 2 for a, b in zip(seps, seps[1:])):
            yield list(seps)


def relerr(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


# ---------------------------------------------------------------- building blocks

def test_gepp_matches_lapack():
    rng = np.random.default_rng(11)
    for n in (1, 2, 5, 17, 40):
        Ad = rng.standard_normal((n, n))
        Fd = rng.standard_normal((n, 3))
        X = oracle.gepp_solve(Ad, Fd)
        assert relerr(X, np.linalg.solve(Ad, Fd)) < 1e-12


def test_gepp_needs_pivoting():
    # zero leading entry: elimination without row interchanges breaks down
    Ad = np.array([[0.0, 1.0], [1.0, 1.0]])
    X = oracle.gepp_solve(Ad, np.array([[1.0], [2.0]]))
    assert np.allclose(X[:, 0], [1.0, 1.0], rtol=0, atol=1e-15)
    with pytest.raises(oracle.OracleError):
        oracle.gepp_solve(np.zeros((3, 3)), np.ones((3, 1)))


def test_inverse_matches_lapack_and_pivots():
    rng = np.random.default_rng(12)
    for n in (1, 3, 16, 33):
        D = rng.standard_normal((n, n))
        G = oracle.inverse(D)
        assert relerr(G, np.linalg.inv(D)) < 1e-11
        assert np.abs(G @ D - np.eye(n)).max() < 1e-11
    # a permutation matrix needs row interchanges and inverts exactly to its transpose
    Pm = np.eye(5)[[3, 0, 4, 1, 2]]
    assert np.array_equal(oracle.inverse(Pm), Pm.T)
    with pytest.raises(oracle.OracleError):
        oracle.inverse(np.zeros((4, 4)))


def test_residual_matches_dense_definition():
    A, B, C, F = rand_system(7, 3, 2, seed=5)
    X = np.random.default_rng(6).standard_normal(F.shape)
    r = (F.reshape(-1, 2) - oracle.dense(A, B, C) @ X.reshape(-1, 2))
    want = np.linalg.norm(r, axis=0) / np.linalg.norm(F.reshape(-1, 2), axis=0)
    assert np.allclose(oracle.residual(A, B, C, X, F), want, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- whole solve vs dense

@pytest.mark.parametrize("N,M,R", [(1, 3, 1), (2, 2, 2), (5, 1, 1), (9, 2, 1), (8, 4, 3)])
def test_ta_matches_dense(N, M, R):
    A, B, C, F = rand_system(N, M, R, seed=N * 10 + M)
    assert relerr(oracle.ta_solve(A, B, C, F), dense_solve(A, B, C, F)) < 1e-13


@pytest.mark.parametrize("N,M", [(3, 1), (5, 2), (7, 1), (8, 3), (9, 2)])
def test_dm_every_separator_set_matches_dense(N, M):
    """Brute force: every P and every valid separator set, depth 0 and 1."""
    A, B, C, F = rand_system(N, M, 2, seed=100 + N)
    ref = dense_solve(A, B, C, F)
    n_cases = 0
    for P in range(1, (N + 1) // 2 + 1):
        for seps in all_separator_sets(N, P):
            for depth in (0, 1):
                X = oracle.dm_solve(A, B, C, F, P, seps=seps, depth=depth)
                assert relerr(X, ref) < 1e-13, (P, seps, depth)
                n_cases += 1
    assert n_cases > 0


def test_dm_depth2_matches_dense():
    A, B, C, F = rand_system(200, 2, 2, seed=3)
    ref = dense_solve(A, B, C, F)
    for P, depth in ((40, 1), (40, 2), (64, 2), (99, 3)):
        assert relerr(oracle.dm_solve(A, B, C, F, P, depth=depth), ref) < 1e-13


def test_dm_p1_is_ta_bitwise():
    A, B, C, F = rand_system(13, 4, 2, seed=9)
    assert np.array_equal(oracle.dm_solve(A, B, C, F, 1), oracle.ta_solve(A, B, C, F))


def test_dm_independent_of_partition_on_small_workload():
    A, B, C, F = inputs.cfg_small()
    ref = oracle.ta_solve(A, B, C, F)
    for P in (2, 4, 7, 16, 32):
        for depth in (0, 1, 2):
            X = oracle.dm_solve(A, B, C, F, P, depth=depth)
            assert relerr(X, ref) < 1e-14
            assert oracle.residual(A, B, C, X, F).max() < 1e-14


# ---------------------------------------------------------------- closed forms (M = 1)

def laplace1d(N, R=1):
    A = np.full((N, 1, 1), 2.0)
    B = np.full((N, 1, 1), -1.0)
    C = np.full((N, 1, 1), -1.0)
    F = np.ones((N, 1, R))
    return A, B, C, F


@pytest.mark.parametrize("N", [1, 2, 7, 64, 1001])
def test_manufactured_solution_ta(N):
    A, B, C, F = laplace1d(N)
    i = np.arange(1, N + 1)
    exact = i * (N + 1 - i) / 2.0
    X = oracle.ta_solve(A, B, C, F)
    assert np.abs(X[:, 0, 0] - exact).max() <= 1e-12 * exact.max()


def test_ta_auxiliaries_closed_form():
    N = 12
    A, B, C, F = laplace1d(N)
    X, aux = oracle.dm_solve(A, B, C, F, 1, want_aux=True)
    i = np.arange(1, N + 1)
    assert np.allclose(aux["D"][:, 0, 0], (i + 1) / i, rtol=1e-15, atol=0)
    assert np.allclose(aux["E"][:-1, 0, 0], -i[:-1] / (i[:-1] + 1), rtol=1e-15, atol=0)


def test_spikes_and_coupling_closed_form():
    N, P = 40, 5
    A, B, C, F = laplace1d(N)
    seps = [6, 15, 21, 33]          # unequal subsystems of 6, 8, 5, 11, 6 rows
    X, aux = oracle.dm_solve(A, B, C, F, P, seps=seps, want_aux=True)
    bounds = [-1] + seps + [N]
    sizes = []
    for k in range(P):
        r, e = bounds[k] + 1, bounds[k + 1] - 1
        n = e - r + 1
        sizes.append(n)
        loc = np.arange(1, n + 1)
        if k > 0:
            assert np.allclose(aux["ZL"][r:e + 1, 0, 0], -(n + 1 - loc) / (n + 1), rtol=1e-14, atol=0)
        if k < P - 1:
            assert np.allclose(aux["ZR"][r:e + 1, 0, 0], -loc / (n + 1), rtol=1e-14, atol=0)
    for j in range(P - 1):
        a, b = sizes[j] + 1, sizes[j + 1] + 1
        assert abs(aux["Hd"][j, 0, 0] - (1 / a + 1 / b)) < 1e-15
        if j > 0:
            assert abs(aux["Hb"][j, 0, 0] + 1 / a) < 1e-15
        if j < P - 2:
            assert abs(aux["Hc"][j, 0, 0] + 1 / b) < 1e-15
    i = np.arange(1, N + 1)
    assert np.abs(X[:, 0, 0] - i * (N + 1 - i) / 2).max() < 1e-11


# ---------------------------------------------------------------- structured special cases

def test_kronecker_case_decouples_into_scalar_problems():
    rng = np.random.default_rng(21)
    N, M, R, P = 30, 4, 2, 4
    a = 3.0 + rng.uniform(size=N)
    b = rng.uniform(-1, 1, N)
    c = rng.uniform(-1, 1, N)
    I = np.eye(M)
    A, B, C = a[:, None, None] * I, b[:, None, None] * I, c[:, None, None] * I
    F = rng.standard_normal((N, M, R))
    X = oracle.dm_solve(A, B, C, F, P, depth=1)
    for comp in range(M):
        xs = oracle.dm_solve(a[:, None, None], b[:, None, None], c[:, None, None],
                             F[:, comp:comp + 1, :], P, depth=1)
        assert np.allclose(X[:, comp, :], xs[:, 0, :], rtol=1e-14, atol=1e-15)


def test_block_diagonal_case():
    rng = np.random.default_rng(22)
    N, M, R, P = 11, 3, 2, 3
    A = rng.standard_normal((N, M, M)) + 4 * np.eye(M)
    Z = np.zeros_like(A)
    F = rng.standard_normal((N, M, R))
    X, aux = oracle.dm_solve(A, Z, Z, F, P, want_aux=True)
    assert np.allclose(X, np.linalg.solve(A, F), rtol=1e-13, atol=1e-14)
    assert not aux["ZL"].any() and not aux["ZR"].any()
    seps = oracle.partition(N, P)
    assert np.array_equal(aux["Hd"], A[seps])


def test_singular_block_is_reported():
    A, B, C, F = rand_system(9, 2, 1, seed=4)
    A[4] = 0.0
    B[4] = 0.0
    C[3] = 0.0  # row 4 of D becomes exactly zero at the first step
    with pytest.raises(oracle.OracleError) as ei:
        oracle.dm_solve(A, B, C, F, 1)
    assert ei.value.row == 4


# ---------------------------------------------------------------- partition rules

def test_partition_rule():
    assert oracle.partition(64, 4) == [16, 32, 48]      # subsystems 16, 15, 15, 15
    for N in range(1, 60):
        for P in range(1, (N + 1) // 2 + 1):
            seps = oracle.partition(N, P)
            bounds = [-1] + seps + [N]
            sizes = [bounds[k + 1] - bounds[k] - 1 for k in range(P)]
            assert sum(sizes) == N - (P - 1) and min(sizes) >= 1
            assert max(sizes) - min(sizes) <= 1 and sizes == sorted(sizes, reverse=True)
    with pytest.raises(ValueError):
        oracle.partition(6, 4)


def test_balanced_partition_rule():
    """Sec. 5.1, second case (Eq. SpeedupMPNk): end subsystems alpha and beta times the middle
    ones, N_k = (N - (P-1)) / (P - 2 + alpha + beta), in whole rows."""
    for N in range(3, 120, 7):
        for P in range(2, (N + 1) // 2 + 1):
            for a, b in ((7 / 4, 7 / 6), (1.0, 1.0), (3.0, 1.5)):
                seps = oracle.balanced_partition(N, P, a, b)
                bounds = [-1] + seps + [N]
                n = [bounds[k + 1] - bounds[k] - 1 for k in range(P)]
                assert sum(n) == N - (P - 1) and min(n) >= 1
                x = (N - P + 1) / (P - 2 + a + b)
                if P > 2:
                    assert max(n[1:-1]) - min(n[1:-1]) <= 1
                    if x * min(a, b) >= 1 and N - P + 1 - round(a * x) - round(b * x) >= P - 2:
                        assert abs(n[0] - a * x) <= 0.5 + 1e-9 and abs(n[-1] - b * x) <= 0.5 + 1e-9
                if a == b == 1.0:
                    assert max(n) - min(n) <= 1 + (P == 2)
    # the paper's validation size (N = 3071 block rows), P = 16: middle size
    # (3071 - 15) / (14 + 7/4 + 7/6) = 180.7
    seps = oracle.balanced_partition(3071, 16)
    bounds = [-1] + seps + [3071]
    n = [bounds[k + 1] - bounds[k] - 1 for k in range(16)]
    assert n[0] == 316 and n[-1] == 211 and set(n[1:-1]) <= {180, 181}
    with pytest.raises(ValueError):
        oracle.balanced_partition(6, 4)


def test_default_m_rule():
    # Eq. SuppMatrM for P >= 21, boundary m = P/3 below, at least 2
    assert oracle.default_m(3, 16, 1) == 1
    assert oracle.default_m(8, 128, 4) == 2
    assert oracle.default_m(512, 128, 4) == 34
    for P in range(4, 600):
        m = oracle.default_m(P, 64, 1)
        assert 2 <= m <= max(2, P // 3) and 2 * m - 1 <= P - 1


# ---------------------------------------------------------------- operation counts (Sec. 4)

@pytest.mark.parametrize("N", [1, 2, 5, 40])
def test_counter_ta_table1(N):
    A, B, C, F = rand_system(N, 2, 1, seed=1)
    cnt = oracle.Counter()
    oracle.ta_solve(A, B, C, F, counter=cnt)
    _, total = costmodel.ta_table1(N)
    assert (cnt.inv + cnt.mm, cnt.mr) == total
    assert cnt.inv == N


@pytest.mark.parametrize("N,P,seps", [(9, 2, None), (31, 4, None), (40, 5, [6, 15, 21, 33]),
                                      (57, 7, None), (41, 3, [1, 39])])
def test_counter_dm_total(N, P, seps):
    A, B, C, F = rand_system(N, 2, 1, seed=2)
    cnt = oracle.Counter()
    oracle.dm_solve(A, B, C, F, P, seps=seps, counter=cnt)
    s = seps or oracle.partition(N, P)
    bounds = [-1] + s + [N]
    Nks = [bounds[k + 1] - bounds[k] - 1 for k in range(P)]
    assert (cnt.inv + cnt.mm, cnt.mr) == costmodel.dm_total(Nks)
    # Tab. 2 row by row adds up to the same total
    rows = [costmodel.dm_table2_subsystem(k, P, Nk) for k, Nk in enumerate(Nks, 1)]
    rows += [costmodel.dm_table2_coupling_products(k, P) for k in range(1, P + 1)]
    rows += [costmodel.dm_table2_recovery(k, P, Nk) for k, Nk in enumerate(Nks, 1)]
    rows += [(3 * P - 5, 3 * P - 5)]
    assert tuple(map(sum, zip(*rows))) == costmodel.dm_total(Nks)


@pytest.mark.parametrize("N,P", [(63, 16), (120, 21), (300, 40)])
def test_counter_dm_rec1(N, P):
    A, B, C, F = rand_system(N, 2, 1, seed=3)
    cnt = oracle.Counter()
    oracle.dm_solve(A, B, C, F, P, depth=1, counter=cnt)
    s = oracle.partition(N, P)
    bounds = [-1] + s + [N]
    Nks = [bounds[k + 1] - bounds[k] - 1 for k in range(P)]
    m = oracle.default_m(P, 2, 1)
    sc = oracle.partition(P - 1, m)
    cb = [-1] + sc + [P - 1]
    Mjs = [cb[j + 1] - cb[j] - 1 for j in range(m)]
    assert (cnt.inv + cnt.mm, cnt.mr) == costmodel.dm_rec1(Nks, Mjs)


# ---------------------------------------------------------------- cost model

def test_costmodel_printed_example():
    with open(os.path.join(GOLD, "costmodel_example.json")) as f:
        g = json.load(f)
    M, J, m = costmodel.p3dmrec4(g["N"], g["n"], g["l"])
    assert (round(M), round(J), round(m)) == (g["M"], g["J"], g["m"])


def _weighted(cnt, n, l):
    """A count of the operation counter in multiplicative operations for block
    size n and l right-hand-side columns (Sec. 4 units)."""
    return (cnt["inv"] + cnt["mm"]) * n**3 + cnt["mr"] * n**2 * l


def _count_ta(N):
    A, B, C, F = rand_system(N, 2, 1, seed=50 + N)
    cnt = oracle.Counter()
    oracle.ta_solve(A, B, C, F, counter=cnt)
    return cnt.as_dict()


def _count_dm(sizes):
    """Operation counter of the method on a system with the given subsystem sizes."""
    P = len(sizes)
    seps, pos = [], 0
    for x in sizes[:-1]:
        pos += x
        seps.append(pos)
        pos += 1
    N = sum(sizes) + P - 1
    A, B, C, F = rand_system(N, 2, 1, seed=60 + N)
    cnt = oracle.Counter()
    oracle.dm_solve(A, B, C, F, P, seps=seps, counter=cnt)
    return cnt.as_dict()


def _serial_middle(Nk, n, l):
    """Multiplicative operations of one middle subsystem of Nk rows (its
    solve of Eq. e231, its share of the coupling products and of the
    recovery), taken from the operation counter: a method run with
    subsystems (2, Nk, 3) minus a run with (2, 3) counts the middle subsystem
    plus the growth of the coupling Thomas algorithm from one to two rows."""
    w3 = _weighted(_count_dm([2, Nk, 3]), n, l)
    w2 = _weighted(_count_dm([2, 3]), n, l)
    return w3 - w2 - (_weighted(_count_ta(2), n, l) - _weighted(_count_ta(1), n, l))


@pytest.mark.parametrize("n,l", [(400, 1), (100, 37), (3, 8)])
def test_speedup_mp_matches_counted_operations(n, l):
    """Eq. SpeedupMP is the Thomas algorithm's operations over the serial
    operations of the method with P equal subsystems: one middle subsystem
    plus the coupling system of P-1 rows by the Thomas algorithm (Sec. 5.1).
    Both are built from the operation counter (pinned to Tab. 1 and Tab. 2);
    n and l enter with different powers, so a swapped l/n fails."""
    for Nk, P in [(4, 3), (7, 5), (12, 9), (30, 17)]:
        N = P * Nk + P - 1
        ta = _weighted(_count_ta(N), n, l)
        serial = _serial_middle(Nk, n, l) + _weighted(_count_ta(P - 1), n, l)
        assert np.isclose(costmodel.speedup_mp(N, P, n, l), ta / serial, rtol=1e-13, atol=0)
    N = 3071
    for P in range(2, 300):
        assert costmodel.speedup_mp(N, P, n, l) > costmodel.speedup_mp_lower(N, P)
    # linear growth S ~ 3P/7 for P << N and l << n, as stated after Eq. SpeedupMP
    assert np.isclose(costmodel.speedup_mp(10**9, 10, 10**6, 1) / (3 * 10 / 7), 1.0, rtol=1e-4)


def test_speedup_maximiser_is_the_counted_optimum():
    """Eq. MAXSpeedP is the maximiser of Eq. SpeedupMP (checked on a fine
    grid of real P) and reduces to sqrt(7(N+1)/3) for l << n (Sec. 5.1)."""
    N = 3071
    for n, l in [(400, 1), (100, 100), (50, 400)]:
        Popt = costmodel.speedup_optimal_P(N, n, l)
        grid = np.linspace(2.0, 600.0, 600001)
        best = grid[np.argmax(costmodel.speedup_mp(N, grid, n, l))]
        assert abs(best - Popt) < 2e-3
    assert np.isclose(costmodel.speedup_optimal_P(N, 10**9, 1), np.sqrt(7 * (N + 1) / 3), rtol=1e-8)


@pytest.mark.parametrize("n,l", [(400, 1), (64, 64), (16, 200)])
def test_suppmatr_m_minimises_counted_operations(n, l):
    """Eq. SuppMatrM minimises the serial operations of Eq. DMrec2: a middle
    subsystem of N1 rows, a middle coupling subsystem of (P-m)/m rows and the
    Thomas algorithm on the m-1 separators of the coupling system.  Every
    term is taken from the operation counter; a middle subsystem's count is
    linear in its rows (checked), so it extends to fractional sizes."""
    per_row = _serial_middle(1, n, l)
    for Nk in (2, 5, 11):
        assert _serial_middle(Nk, n, l) == Nk * per_row
    ta = {k: _weighted(_count_ta(k), n, l) for k in (1, 2)}
    ta_row = ta[2] - ta[1]                 # Tab. 1: (3k-2) is linear in k
    for P in (30, 64, 256, 1000):
        m = np.linspace(2.0, P / 3.0, 200001)
        serial = ((P - m) / m) * per_row + (ta[1] + (m - 2) * ta_row)
        best = m[np.argmin(serial)]
        assert abs(best - costmodel.suppmatr_m(P, n, l)) < 1e-2 * max(1.0, best / 10)
    # the statements that follow Eq. SuppMatrM: m ~ sqrt(7P/3) for l << n,
    # and the requirement (P-m)/m >= 2 holds exactly from P = 21 on
    assert np.isclose(costmodel.suppmatr_m(300, 10**9, 1), np.sqrt(7 * 300 / 3), rtol=1e-8)
    assert np.isclose(3 * costmodel.suppmatr_m(21, 10**9, 0), 21.0, rtol=1e-12)
    assert 3 * costmodel.suppmatr_m(20, 10**9, 0) > 20.0


# ---------------------------------------------------------------- recursion into the subsystems

def _sizes(N, P):
    b = [-1] + oracle.partition(N, P) + [N]
    return [b[k + 1] - b[k] - 1 for k in range(P)]


@pytest.mark.parametrize("N,P,J,depth", [(40, 3, 2, 0), (63, 4, 3, 0), (90, 5, 4, 0), (121, 6, 2, 0), (70, 2, 5, 0),
                                         (200, 12, 3, 1)])
def test_subsystem_recursion_matches_dense_and_counts(N, P, J, depth):
    """Every subsystem solved by the DM with J sub-subsystems (Sec. 4.2.2):
    the solution of the dense system, the same outer coupling system as the
    plain method (it is the Schur complement onto the separator rows, however
    the subsystems are solved), and the operation counter equal to Eqs.
    DMrec121 (first subsystem), DMrec1212 (last) and DMrec122 (the others)
    plus the coupling products and recovery of Tab. 2 and the coupling
    system (Thomas algorithm, or Eq. DMrec1 with depth 1)."""
    A, B, C, F = rand_system(N, 2, 2, seed=70 + N)
    cnt = oracle.Counter()
    X, aux = oracle.dm_solve(A, B, C, F, P, depth=depth, J=J, counter=cnt, want_aux=True)
    assert relerr(X, dense_solve(A, B, C, F)) < 1e-13
    X0, aux0 = oracle.dm_solve(A, B, C, F, P, depth=depth, want_aux=True)
    for name in ("Hd", "Hb", "Hc", "fhat", "h"):
        assert np.allclose(aux[name], aux0[name], rtol=1e-12, atol=1e-13), name
    Ls = [_sizes(nk, J) for nk in _sizes(N, P)]
    coupling = None
    if depth:
        m = oracle.default_m(P, 2, 2)
        coupling = costmodel.dm_total(_sizes(P - 1, m))
    assert (cnt.inv + cnt.mm, cnt.mr) == costmodel.dm_total_subrec(Ls, coupling)


def test_subsystem_recursion_j1_is_the_plain_method():
    A, B, C, F = rand_system(50, 3, 1, seed=80)
    assert np.array_equal(oracle.dm_solve(A, B, C, F, 4, J=1), oracle.dm_solve(A, B, C, F, 4))


def test_dmrec3_optimum_is_the_quartic_root():
    """Eq. P3DMrec3 (J, with M from Eq. P2DMrec3) is the minimiser of Eq.
    DMrec3 over real M and J (P = M J free) on a grid, for the parameters of
    the paper's figures and others."""
    for N, n, l in [(3071, 400, 1), (3071, 100, 1), (4095, 256, 64), (2047, 128, 4)]:
        M, J = costmodel.p3dmrec3(N, n, l)
        Ms = np.linspace(0.5 * M, 1.5 * M, 801)[:, None]
        Js = np.linspace(0.5 * J, 1.5 * J, 801)[None, :]
        f = costmodel.dmrec3(N, Ms, Js, n, l)
        i, j = np.unravel_index(np.argmin(f), f.shape)
        assert abs(Ms[i, 0] - M) / M < 3e-3 and abs(Js[0, j] - J) / J < 3e-3, (N, n, l, M, J, Ms[i, 0], Js[0, j])
