"""GPU: mixed precision with iterative refinement (BTD_PREC_F32_REFINE).
The products of the top level's factor sweeps run on FP32 MFMA with FP32
accumulation; the solve with those factors is FP32-accurate, and the
refinement (FP64 residual, correction and coupling systems) brings it to
the FP64 bar against the FP64 oracle.  The error of each precision against
the oracle is printed per case.
"""
import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, col_relerr, require_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL_X = 1e-10
TOL_RES = 1e-12


@pytest.mark.parametrize("kind,N,M,R,P,depth", [
    ("diag", 200, 64, 3, 16, 1),
    ("diag", 120, 256, 1, 8, 1),
    ("diag", 97, 100, 20, 9, 0),
    ("large_like", 300, 256, 2, 20, 2),
    ("faddeev", 256, 32, 2, 16, 1),
])
def test_refined_solve_matches_oracle(kind, N, M, R, P, depth):
    torch = require_gpu()
    print(f"case mixed {kind} N={N} M={M} R={R} P={P} depth={depth}", flush=True)
    if kind == "diag":
        A, B, C, F = inputs.diag_dominant(N, M, R, seed=1200 + N)
    elif kind == "large_like":
        A, B, C, F = inputs.diag_dominant(N, M, R, seed=1201, shift=1.5)
    else:
        A, B, C, F = inputs.faddeev_like(N, M, R, seed=1202)
    Xo = oracle.dm_solve(A, B, C, F, P, depth=depth)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=depth, max_nrhs=R, prec="f32_refine")
    X32 = plan.solve(Fd).cpu().numpy()
    assert plan.info() == (0, -1, -1)
    err32 = col_relerr(X32, Xo)
    # the products really ran in FP32: the unrefined error is far above FP64 rounding
    assert 1e-11 < err32 < 1e-2, err32
    max_iter = 30 if kind == "faddeev" else 5
    X, iters, res = plan.solve_refine(Fd, tol=TOL_RES, max_iter=max_iter)
    Xr = X.cpu().numpy()
    err = col_relerr(Xr, Xo)
    print(f"  unrefined error {err32:.2e}; refined after {iters} corrections: error {err:.2e}, residual {res:.2e}",
          flush=True)
    assert iters >= 1 and res <= TOL_RES
    assert_parity(Xr, Xo, TOL_X)
    assert oracle.residual(A, B, C, Xr, F).max() <= TOL_RES
    plan.destroy()


def test_fp64_plan_needs_no_correction_and_status():
    """An FP64 plan meets the tolerance with its first solve; an FP32 plan
    with no correction allowed reports BTD_ERR_NOT_CONVERGED; NaN in F is
    reported by the solve check and does not converge."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(80, 48, 2, seed=1210)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    p64 = btd.factor(Ad, Bd, Cd, P=8, depth=1, max_nrhs=2)
    X, iters, res = p64.solve_refine(Fd, tol=1e-12)
    assert iters == 0 and res <= 1e-12
    assert_parity(X.cpu().numpy(), oracle.dm_solve(A, B, C, F, 8, depth=1), TOL_X)
    p32 = btd.factor(Ad, Bd, Cd, P=8, depth=1, max_nrhs=2, prec="f32_refine")
    with pytest.raises(btd.BtdError) as e:
        p32.solve_refine(Fd, tol=1e-12, max_iter=0)
    assert e.value.code == btd.BTD_ERR_NOT_CONVERGED
    Fb = F.copy()
    Fb[3, 7, 1] = np.nan
    with pytest.raises(btd.BtdError) as e:
        p32.solve_refine(to_dev(torch, Fb)[0], tol=1e-12, max_iter=3)
    assert e.value.code == btd.BTD_ERR_NOT_CONVERGED
    assert p32.solve_info() == (btd.BTD_ERR_NONFINITE, 3, 1)
    p64.destroy()
    p32.destroy()
