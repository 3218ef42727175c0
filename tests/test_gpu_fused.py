"""GPU: btd_factor_solve (factor and solve in one call, each level's
right-hand side swept on a side stream while the level's spikes and the
deeper levels are factored) against btd_factor followed by btd_solve.

The two run the same kernels on the same data in the same order per
buffer; only the overlap between streams differs, so the solutions and the
factors must agree BIT FOR BIT.  One case per configuration is also checked
against the FP64 oracle, and a captured graph of the fused call is replayed
against its eager result.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, require_gpu, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # N, M, R, P, depth, coupling_rows, sub_parts
    (1, 16, 1, 1, 0, 0, 0),          # one block row, TA only
    (40, 33, 3, 6, 0, 0, 0),         # one level of P > 1, ragged M
    (80, 16, 2, 16, 1, 0, 0),        # two chunk groups, coupling recursion
    (300, 32, 5, 40, 2, 0, 0),       # three levels
    (257, 64, 8, 24, 1, 4, 0),       # coupling_rows split, ragged N
    (150, 16, 3, 8, 1, 0, 3),        # recursion into the subsystems
    (96, 130, 2, 8, 1, 0, 0),        # M above 128 (other tile shapes)
]


@pytest.mark.parametrize("N,M,R,P,depth,crow,J", CASES)
def test_fused_bit_identical(N, M, R, P, depth, crow, J):
    torch = require_gpu()
    print(f"case fused N={N} M={M} R={R} P={P} depth={depth} crow={crow} J={J}", flush=True)
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=1100 + N)
    F2 = inputs.diag_dominant(N, M, R, seed=1200 + N)[3]
    Ad, Bd, Cd, Fd, F2d = to_dev(torch, A, B, C, F, F2)
    kw = dict(P=P, depth=depth, max_nrhs=R, coupling_rows=crow, sub_parts=J)
    ref = btd.factor(Ad, Bd, Cd, **kw)
    X_ref = ref.solve(Fd)
    fused, X = btd.factor_solve(Ad, Bd, Cd, Fd, **kw)
    torch.cuda.synchronize()
    assert fused.info() == (0, -1, -1)
    assert fused.solve_info() == (0, -1, -1)
    assert torch.equal(X, X_ref)
    # same factors: a later solve with either plan is the same
    assert torch.equal(fused.solve(F2d), ref.solve(F2d))
    Xn = X.cpu().numpy()
    assert_parity(Xn, oracle.dm_solve(A, B, C, F, P, depth=depth, J=max(J, 1)), 1e-10)
    ref.destroy()
    fused.destroy()


def test_fused_in_place_and_nonfinite():
    """X == F (in place) gives the same solution; a non-finite entry of F is
    reported by the fused call's solve check as by btd_solve's."""
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(90, 24, 3, seed=1301)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    ref = btd.factor(Ad, Bd, Cd, P=12, depth=1, max_nrhs=3)
    X_ref = ref.solve(Fd)
    Fi = Fd.clone()
    fused, X = btd.factor_solve(Ad, Bd, Cd, Fi, X=Fi, P=12, depth=1)
    torch.cuda.synchronize()
    assert X.data_ptr() == Fi.data_ptr()
    assert torch.equal(X, X_ref)
    fused.destroy()
    Fb = F.copy()
    Fb[40, 3, 1] = np.nan
    fused, _ = btd.factor_solve(Ad, Bd, Cd, to_dev(torch, Fb)[0], P=12, depth=1)
    assert fused.solve_info() == (btd.BTD_ERR_NONFINITE, 40, 1)
    assert fused.info() == (0, -1, -1)
    fused.destroy()
    ref.destroy()


def test_fused_rejects_small_solve_workspace():
    torch = require_gpu()
    A, B, C, F = inputs.diag_dominant(40, 8, 2, seed=1302)
    Ad, Bd, Cd, Fd = to_dev(torch, A, B, C, F)
    d, _keep = btd.make_desc(40, 8, 4, 0, 2)
    fb, sb = btd.workspace_bytes(40, 8, 4, 0, 2)
    fws, fptr = btd._aligned_buffer(fb, Ad.device)
    sws, sptr = btd._aligned_buffer(sb, Ad.device)
    X = torch.empty_like(Fd)
    h = ctypes.c_void_p()
    L = btd.lib()
    args = (ctypes.byref(d), Ad.data_ptr(), Bd.data_ptr(), Cd.data_ptr(), fptr, fb, 2, Fd.data_ptr(), X.data_ptr())
    assert L.btd_factor_solve(*args, None, sb, None, ctypes.byref(h)) == -11
    assert L.btd_factor_solve(*args, sptr + 8, sb, None, ctypes.byref(h)) == -11
    assert L.btd_factor_solve(*args, sptr, sb - 256, None, ctypes.byref(h)) == -12
    assert not h.value
    torch.cuda.synchronize()
