"""GPU: btd_solve_noalloc (the solve without a workspace argument, scratch in
the library's static device array) against btd_solve through the C ABI:
the same kernels and arithmetic, so the results must agree bit for bit.
Two calls in a row, the second with a smaller system and fewer columns
(the static array keeps the first call's contents), and the host-side
rejection of a solve whose scratch exceeds the array.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _solve_both(torch, A, B, C, F, P, depth, max_nrhs, R):
    L = btd.lib()
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    Fd = to_dev(torch, F[:, :, :R])[0]
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=depth, max_nrhs=max_nrhs)
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    X_ref = torch.full_like(Fd, np.nan)
    ws, ptr = btd._aligned_buffer(plan.solve_bytes, Ad.device)
    assert L.btd_solve(plan.handle, R, Fd.data_ptr(), X_ref.data_ptr(), ptr, plan.solve_bytes, sh) == 0
    X_na = torch.full_like(Fd, np.nan)
    assert L.btd_solve_noalloc(plan.handle, R, Fd.data_ptr(), X_na.data_ptr(), sh) == 0
    torch.cuda.synchronize()
    assert plan.info() == (0, -1, -1)
    out = X_ref.cpu().numpy(), X_na.cpu().numpy()
    plan.destroy()
    return out


def test_noalloc_matches_solve_two_calls():
    torch = require_gpu()
    print("case noalloc: N=300 M=48 P=16 depth=2 R=8, then N=100 M=32 P=8 depth=1 R=2", flush=True)
    A, B, C, F = inputs.diag_dominant(300, 48, 8, seed=901)
    X_ref, X_na = _solve_both(torch, A, B, C, F, 16, 2, 8, 8)
    assert np.array_equal(X_ref, X_na)
    assert_parity(X_na, oracle.dm_solve(A, B, C, F, 16, depth=1), 1e-10)
    # second call: smaller system and fewer columns than the plan allows
    A, B, C, F = inputs.diag_dominant(100, 32, 4, seed=902)
    X_ref, X_na = _solve_both(torch, A, B, C, F, 8, 1, 4, 2)
    assert np.array_equal(X_ref, X_na)
    assert_parity(X_na, oracle.dm_solve(A, B, C, np.ascontiguousarray(F[:, :, :2]), 8, depth=1), 1e-10)


def test_noalloc_rejects_oversized_scratch():
    """A solve whose scratch exceeds the static array is rejected on the host
    with BTD_ERR_SCRATCH (nothing enqueued, X untouched); the same plan with
    fewer columns fits."""
    torch = require_gpu()
    N, M, P = 64, 16, 16
    Rbig = 40000
    _, sb = btd.workspace_bytes(N, M, P, 1, Rbig)
    assert sb > btd.NOALLOC_SCRATCH_BYTES
    A, B, C, _ = inputs.diag_dominant(N, M, 1, seed=903)
    Ad, Bd, Cd = to_dev(torch, A, B, C)
    plan = btd.factor(Ad, Bd, Cd, P=P, depth=1, max_nrhs=Rbig)
    F = torch.zeros((N, M, Rbig), dtype=torch.float64, device="cuda")
    X = torch.full_like(F, 7.0)
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = btd.lib()
    assert L.btd_solve_noalloc(plan.handle, Rbig, F.data_ptr(), X.data_ptr(), sh) == btd.BTD_ERR_SCRATCH
    torch.cuda.synchronize()
    assert bool((X == 7.0).all())
    assert L.btd_solve_noalloc(plan.handle, 3, F.data_ptr(), X.data_ptr(), sh) == 0
    torch.cuda.synchronize()
    assert bool((X.reshape(-1)[: N * M * 3] == 0).all())   # X = A^{-1} 0 = 0, as [N][M][3] in the first values
    assert bool((X.reshape(-1)[N * M * 3:] == 7.0).all())
    assert L.btd_solve_noalloc(None, 1, F.data_ptr(), X.data_ptr(), sh) == -1
    assert L.btd_solve_noalloc(plan.handle, 0, F.data_ptr(), X.data_ptr(), sh) == -2
    plan.destroy()
