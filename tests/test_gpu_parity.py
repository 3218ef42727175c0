"""GPU parity: the HIP decomposition-method path (through the C ABI) against
the FP64 CPU oracle, on the same seeded inputs.

Bar (FP64): max over RHS columns of ||X - X_oracle||_2 / ||X_oracle||_2 <=
1e-10, every element within 1e-10 of the column's largest magnitude, and the
relative residual ||F - A X||_2 / ||F||_2 <= 1e-12 per column.
"""
import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, col_relerr, require_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL_X = 1e-10
TOL_RES = 1e-12


def run_gpu(torch, A, B, C, F, P, depth=0, seps=None, max_nrhs=None, inplace=False, coupling_rows=0):
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    R = F.shape[2]
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=depth, max_nrhs=max_nrhs or R, seps=seps,
                      coupling_rows=coupling_rows)
    Xd = plan.solve(Fd, Fd if inplace else None)
    st = plan.info()
    assert st == (0, -1, -1), st
    X = Xd.cpu().numpy()
    Fd2 = to_dev(torch, F)[0]
    res = btd.residual(Ad, Bd, Cd, Xd, Fd2).cpu().numpy()
    plan.destroy()
    return X, res


def check_case(torch, A, B, C, F, P, depth=0, seps=None, inplace=False, coupling_rows=0):
    print(f"case N={A.shape[0]} M={A.shape[1]} R={F.shape[2]} P={P} depth={depth} seps={seps} "
          f"coupling_rows={coupling_rows}", flush=True)
    X, res_gpu = run_gpu(torch, A, B, C, F, P, depth, seps, inplace=inplace, coupling_rows=coupling_rows)
    Xo = oracle.dm_solve(A, B, C, F, P, seps=seps, depth=depth)
    assert_parity(X, Xo, TOL_X)
    res = oracle.residual(A, B, C, X, F)
    assert res.max() <= TOL_RES, res
    assert res_gpu.max() <= TOL_RES, res_gpu
    return X


@pytest.mark.parametrize("N,M,R", [(1, 4, 1), (9, 16, 3), (64, 33, 2), (5, 256, 1),
                                   (1, 16, 8), (9, 16, 8), (5, 256, 64), (7, 33, 70), (3, 130, 9)])
def test_residual_kernel_matches_oracle(N, M, R):
    """The device residual of a perturbed solution (residual well above
    rounding) against the oracle's residual of the same X (R >= 2 takes the
    MFMA tile kernel, one column the row kernel).  The perturbation keeps
    ||r|| near 1e-3 ||F||: the rounding of A X (about 3 M u |A||X| per
    element, in either accumulation order) is then near 1e-12 of ||r||, well
    inside the 1e-10 bar."""
    torch = require_gpu()
    A, B, C, F, xs = inputs.diag_dominant(N, M, R, seed=40 + N, want_xstar=True)
    X = xs + 1e-3 * np.random.default_rng(1).standard_normal(xs.shape)
    Ad, Bd, Cd, Xd, Fd = to_dev(torch, A, B, C, X, F)
    res_gpu = btd.residual(Ad, Bd, Cd, Xd, Fd).cpu().numpy()
    res = oracle.residual(A, B, C, X, F)
    assert np.allclose(res_gpu, res, rtol=1e-10, atol=0)


@pytest.mark.parametrize("P,depth", [(1, 0), (2, 0), (4, 0), (7, 0), (4, 1), (16, 1), (32, 1), (32, 2)])
def test_small_workload(P, depth):
    torch = require_gpu()
    A, B, C, F = inputs.cfg_small()
    check_case(torch, A, B, C, F, P, depth)


@pytest.mark.parametrize("N,M,R,P,depth", [
    (1, 5, 1, 1, 0), (2, 3, 2, 1, 0), (3, 1, 1, 2, 0), (5, 1, 3, 3, 0), (13, 17, 1, 5, 0),
    (40, 33, 5, 6, 1), (21, 65, 33, 4, 0), (30, 100, 2, 7, 1), (9, 129, 65, 3, 0), (12, 64, 64, 4, 0),
    (25, 31, 7, 12, 1), (9, 257, 3, 3, 1), (6, 300, 20, 2, 0), (10, 256, 1, 4, 0),
])
def test_ragged_shapes(N, M, R, P, depth):
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=1000 + N * 7 + M)
    check_case(torch, A, B, C, F, P, depth)


def test_max_block_size():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(7, btd.BTD_MAX_M, 2, seed=77)
    check_case(torch, A, B, C, F, 3, 0)


@pytest.mark.parametrize("N,M,P,depth", [(200, 24, 8, 0), (301, 40, 12, 1)])
def test_balanced_partition(N, M, P, depth):
    """The balanced partition of Sec. 4 (longer first and last subsystems)."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(N, M, 2, seed=600 + N)
    check_case(torch, A, B, C, F, P, depth, seps=btd.balanced_separators(N, P))


def test_explicit_unequal_separators():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(40, 8, 2, seed=5)
    check_case(torch, A, B, C, F, 5, 0, seps=[1, 15, 21, 33])
    check_case(torch, A, B, C, F, 5, 1, seps=[6, 8, 21, 38])


def test_inplace_and_repeated_solves():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(50, 24, 6, seed=8)
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=6, depth=1, max_nrhs=6)
    Xo = oracle.dm_solve(A, B, C, F, 6, depth=1)
    # several right-hand-side counts against one resident factorisation
    for R in (6, 1, 3):
        Fd = to_dev(torch, F[:, :, :R])[0]
        X = plan.solve(Fd).cpu().numpy()
        assert_parity(X, oracle.dm_solve(A, B, C, F[:, :, :R].copy(), 6, depth=1), TOL_X)
    Fd = to_dev(torch, F)[0]
    plan.solve(Fd, Fd)
    assert_parity(Fd.cpu().numpy(), Xo, TOL_X)
    plan.destroy()


@pytest.mark.parametrize("N,M,R,P,depth", [(40, 256, 16, 5, 1), (33, 100, 40, 4, 0), (60, 32, 17, 20, 1)])
def test_many_rhs_batched_sweep(N, M, R, P, depth):
    """16 or more right-hand sides (the sweep as batched product and
    triangular-solve steps over all subsystems), out of place, then in place
    with fewer columns than the plan allows."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=500 + N + R)
    check_case(torch, A, B, C, F, P, depth)
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=depth, max_nrhs=R + 3)
    Fd = to_dev(torch, F)[0]
    plan.solve(Fd, Fd)
    assert plan.info() == (0, -1, -1)
    assert_parity(Fd.cpu().numpy(), oracle.dm_solve(A, B, C, F, P, depth=depth), TOL_X)
    plan.destroy()


def test_solve_batch_matches_single_solves():
    torch = require_gpu()
    plans, Fs, refs = [], [], []
    for s, (N, M, R, P) in enumerate([(30, 8, 2, 3), (64, 16, 1, 4), (17, 5, 4, 2)]):
        A, B, C, F = inputs.diag_dominant(N, M, R, seed=300 + s)
        Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
        plans.append(btd.factor(Ad, Bd, Cd, P=P, max_nrhs=R))
        Fs.append(Fd)
        refs.append(oracle.dm_solve(A, B, C, F, P))
    Xs = btd.solve_batch(plans, Fs)
    for X, Xo in zip(Xs, refs):
        assert_parity(X.cpu().numpy(), Xo, TOL_X)
    # with room for three solves side by side: the same numbers, bit for bit
    for lanes in (2, 3):
        Xc = btd.solve_batch(plans, Fs, lanes=lanes)
        for X, Y in zip(Xs, Xc):
            assert torch.equal(X, Y)
    for p in plans:
        p.destroy()


def test_deterministic():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(64, 16, 3, seed=9)
    X1, _ = run_gpu(torch, A, B, C, F, 4, 1)
    X2, _ = run_gpu(torch, A, B, C, F, 4, 1)
    assert np.array_equal(X1, X2)


@pytest.mark.parametrize("coupling_rows,depth", [(1, 8), (2, 4), (3, 2)])
def test_coupling_rows_split(coupling_rows, depth):
    """Coupling systems split into subsystems of about k rows instead of Eq.
    SuppMatrM: same solution (the oracle uses the paper's m)."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(400, 24, 3, seed=41, shift=2.0)
    check_case(torch, A, B, C, F, 64, depth, coupling_rows=coupling_rows)


@pytest.mark.parametrize("N,M,P", [(12, 8, 3), (9, 40, 3), (8, 100, 2), (6, 256, 2), (5, 300, 2)])
def test_pivoting_needed(N, M, P):
    """Diagonal blocks with rows permuted (and a zero leading entry): LU
    without row interchanges would break down, and the pivot rows come in
    scattered order across the panels of the LU."""
    torch = require_gpu()
    rng = np.random.default_rng(31 + M)
    R = 2
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=31 + M)
    perm = rng.permutation(M)
    A = A[:, perm, :].copy()          # row-permuted diagonal blocks: zero-free but far from the diagonal
    A[:, 0, 0] = 0.0
    F = inputs.block_matvec(A, B, C, rng.standard_normal((N, M, R)))
    check_case(torch, A, B, C, F, P, 0)


def test_singular_block_reported():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(20, 4, 1, seed=3)
    A[9] = 0.0
    B[9] = 0.0
    C[8] = 0.0
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=3)
    st, row, col = plan.info()
    assert st == btd.BTD_ERR_SINGULAR and row == 9 and col == 0
    plan.destroy()


def test_nonfinite_block_reported():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(20, 4, 1, seed=4)
    A[13, :, 2] = np.nan
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=2)
    st, row, col = plan.info()
    assert st == btd.BTD_ERR_NONFINITE and row == 13
    plan.destroy()


def test_singular_coupling_row_reported():
    """A zero separator block with decoupled neighbours makes the coupling
    system singular; the row reported is the separator row."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(21, 3, 1, seed=6)
    q = btd.default_separators(21, 3)[1]
    A[q] = 0.0
    B[q] = 0.0
    C[q] = 0.0
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=3)
    st, row, col = plan.info()
    assert st == btd.BTD_ERR_SINGULAR and row == q
    plan.destroy()


# ---------------------------------------------------------------- Faddeev-like banded workload

@pytest.fixture(scope="module")
def faddeev():
    A, B, C, F = inputs.cfg_faddeev()
    Xo = oracle.dm_solve(A, B, C, F, 32, depth=0)
    return A, B, C, F, Xo


@pytest.mark.parametrize("P", [8, 32, 128, 512])
@pytest.mark.parametrize("depth", [0, 1])
def test_faddeev_workload(faddeev, P, depth):
    torch = require_gpu()
    A, B, C, F, Xo = faddeev
    print(f"faddeev P={P} depth={depth}", flush=True)
    X, res_gpu = run_gpu(torch, A, B, C, F, P, depth)
    err = col_relerr(X, Xo)
    assert err <= TOL_X, err
    assert res_gpu.max() <= TOL_RES, res_gpu


# ---------------------------------------------------------------- large dense-block workload

def test_large_workload_full_size():
    """N=4096, M=256, the launch configuration the benchmark times: the
    oracle's residual of the GPU solution and the error against the
    manufactured solution x* (F = A x*)."""
    torch = require_gpu()
    N, M, R = 4096, 256, 1
    A, B, C, F, xs = inputs.diag_dominant(N, M, R, seed=2, shift=1.5, want_xstar=True)
    from bench import DEFAULT_P, DEFAULT_DEPTH, DEFAULT_COUPLING_ROWS
    print(f"large N={N} M={M} P={DEFAULT_P} depth={DEFAULT_DEPTH} coupling_rows={DEFAULT_COUPLING_ROWS}", flush=True)
    X, res_gpu = run_gpu(torch, A, B, C, F, DEFAULT_P, DEFAULT_DEPTH, coupling_rows=DEFAULT_COUPLING_ROWS)
    res = oracle.residual(A, B, C, X, F)
    assert res.max() <= TOL_RES, res
    assert res_gpu.max() <= TOL_RES, res_gpu
    assert col_relerr(X, xs) <= TOL_X
