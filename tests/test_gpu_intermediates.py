"""GPU: the intermediates of the method (Sec. 2) against the oracle's, not
only the solution.  Compared are the quantities that do not depend on the
pivot order: E_i = D_i^{-1} C_i (and the right spikes' seeds), the spikes
Z_L and Z_R (Eq. e231), the coupling blocks Hd, Hb, Hc (Eq. e2311), the
subsystem solutions z and the coupling right-hand side f (first half of the
solve), and the coupling solution h (Eq. e232, at the separator rows of X).
The library's values come through its read-only views of the factor
workspace (btd_plan_level_arrays) and the two halves of a solve
(btd_solve_local, btd_solve_finish).
"""
import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, require_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10


def close(got, want, what):
    """Frobenius-relative and element-wise (scaled by the largest magnitude) agreement."""
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert np.all(np.isfinite(got)), what
    scale = max(np.max(np.abs(want)), 1e-300)
    err = np.max(np.abs(got - want)) / scale
    assert err <= TOL, f"{what}: max element error {err:.2e} of the largest magnitude"
    nrm = np.linalg.norm(want)
    if nrm > 0:
        assert np.linalg.norm(got - want) / nrm <= TOL, what


CASES = [
    ("diag", 60, 24, 3, 6),
    ("diag", 97, 40, 2, 9),
    ("diag", 33, 130, 1, 4),
    ("faddeev", 64, 16, 2, 5),
]


@pytest.mark.parametrize("kind,N,M,R,P", CASES)
def test_intermediates_match_oracle(kind, N, M, R, P):
    torch = require_gpu()
    print(f"case intermediates {kind} N={N} M={M} R={R} P={P}", flush=True)
    if kind == "diag":
        A, B, C, F = inputs.diag_dominant(N, M, R, seed=800 + N)
    else:
        A, B, C, F = inputs.faddeev_like(N, M, R, seed=801)
    Xo, aux = oracle.dm_solve(A, B, C, F, P, depth=0, want_aux=True)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=0, max_nrhs=R)
    assert plan.info() == (0, -1, -1)
    lv = plan.level_arrays(0)
    assert (lv["N"], lv["M"], lv["P"]) == (N, M, P)
    sep = lv["sep"].cpu().numpy()
    assert list(sep[1:-1]) == oracle.partition(N, P) and sep[0] == -1 and sep[-1] == N
    W, Z = lv["W"].cpu().numpy(), lv["Z"].cpu().numpy()

    # rows of every subsystem, with the chunk index
    rows_e, rows_zl, rows_zr = [], [], []
    for k in range(P):
        r, e = sep[k] + 1, sep[k + 1] - 1
        for i in range(r, e + 1):
            if not (k == P - 1 and i == e):
                rows_e.append(i)          # E_i, and the right spike's seed at a last row
            if k >= 1:
                rows_zl.append(i)
            if k <= P - 2:
                rows_zr.append(i)
    close(W[rows_e, :, :M], aux["E"][rows_e], "E")
    close(Z[rows_zl, :, :M], aux["ZL"][rows_zl], "Z_L")
    close(Z[rows_zr, :, M:], aux["ZR"][rows_zr], "Z_R")
    for name in ("Hd", "Hb", "Hc"):
        close(lv[name].cpu().numpy(), aux[name], name)

    # first half of the solve: z on the subsystem rows and the coupling right-hand side
    Xz, Fh = plan.solve_local(Fd)
    torch.cuda.synchronize()
    assert plan.solve_info() == (0, -1, -1)
    chunk_rows = [i for i in range(N) if i not in set(sep[1:-1])]
    close(Xz.cpu().numpy()[chunk_rows], aux["z"][chunk_rows], "z")
    close(Fh.cpu().numpy(), aux["fhat"], "fhat")

    # second half from the oracle's coupling solution h: the oracle's X
    H = to_dev(torch, aux["h"])[0]
    X = plan.solve_finish(H, Xz).cpu().numpy()
    assert_parity(X, Xo, TOL)

    # the whole solve: h at the separator rows
    Xf = plan.solve(Fd).cpu().numpy()
    close(Xf[sep[1:-1]], aux["h"], "h")
    assert_parity(Xf, Xo, TOL)
    plan.destroy()


def test_coupling_levels_are_the_next_systems():
    """With recursion, level l+1's blocks are level l's coupling blocks, and
    its subsystem count is the one the plan reports."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(200, 16, 1, seed=810)
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=40, depth=2, max_nrhs=1)
    parts = plan.level_parts()
    assert parts[0] == 40 and parts[-1] == 1 and len(parts) == 4   # 40, m(40), m(m(40)), Thomas algorithm
    l0, l1 = plan.level_arrays(0), plan.level_arrays(1)
    assert (l1["N"], l1["P"]) == (39, parts[1])
    lib = btd.lib()
    out = btd.LevelArrays()
    assert lib.btd_plan_level_arrays(plan.handle, 1, out) == 0
    assert out.A == l0["Hd"].data_ptr() and out.B == l0["Hb"].data_ptr() and out.C == l0["Hc"].data_ptr()
    assert lib.btd_plan_level_arrays(plan.handle, len(parts), out) == -1
    _, aux = oracle.dm_solve(A, B, C, F, 40, depth=0, want_aux=True)
    torch.cuda.synchronize()
    for name in ("Hd", "Hb", "Hc"):
        close(l0[name].cpu().numpy(), aux[name], name)
    plan.destroy()


@pytest.mark.parametrize("N,M,R,P,J,depth,crow", [(63, 16, 2, 4, 3, 0, 0), (200, 24, 3, 12, 3, 1, 0),
                                                 (500, 64, 1, 8, 8, 1, 1), (150, 33, 4, 5, 4, 0, 0),
                                                 (90, 130, 2, 3, 2, 0, 0), (41, 8, 1, 1, 5, 0, 0)])
def test_subsystem_recursion_matches_oracle(N, M, R, P, J, depth, crow):
    """Recursion into the subsystems (sub_parts J, Sec. 4.2.2; with depth 1
    both recursions): the solution element by element against the oracle's
    literal method (every subsystem solved by the DM with J sub-subsystems),
    the outer coupling system the library forms (its level 2) against the
    plain method's coupling blocks, and the outer separators."""
    torch = require_gpu()
    print(f"case sub_parts N={N} M={M} R={R} P={P} J={J} depth={depth} coupling_rows={crow}", flush=True)
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=820 + N)
    Xo = oracle.dm_solve(A, B, C, F, P, depth=depth, J=J)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=depth, max_nrhs=R, coupling_rows=crow, sub_parts=J)
    parts = plan.level_parts()
    assert parts[0] == P * J and (P == 1 or parts[1] == P), parts
    X = plan.solve(Fd).cpu().numpy()
    assert plan.info() == (0, -1, -1)
    assert_parity(X, Xo, TOL)
    assert oracle.residual(A, B, C, X, F).max() <= 1e-12
    if P > 1:
        assert plan.separators() == oracle.partition(N, P)
        _, aux = oracle.dm_solve(A, B, C, F, P, depth=0, want_aux=True)
        out = btd.LevelArrays()
        assert btd.lib().btd_plan_level_arrays(plan.handle, 2, out) == 0
        assert (out.N, out.M) == (P - 1, M)
        l1 = plan.level_arrays(1)
        for name, ptr in (("Hd", out.A), ("Hb", out.B), ("Hc", out.C)):
            assert l1[name].data_ptr() == ptr
            close(l1[name].cpu().numpy(), aux[name], name)
    plan.destroy()
