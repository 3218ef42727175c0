"""GPU: factor + solve captured into a HIP graph (through torch's graph
capture) and replayed.  Every replay must reproduce the eagerly computed
solution exactly (same kernels, same inputs, fixed reduction orders), with
other eager work and synchronisations between the replays; the solution is
also checked against the FP64 oracle.  The system uses enough subsystems for
the library to split them over its side streams, so the fork and join events
are part of the captured graph.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import btd, inputs
from gpu_util import assert_parity, require_gpu, to_dev

pytestmark = pytest.mark.gpu


class AbiRun:
    """factor + solve through the C ABI with workspaces allocated once."""

    def __init__(self, torch, A, B, C, F, P, depth, fused=False):
        self.torch, self.L, self.fused = torch, btd.lib(), fused
        self.A, self.B, self.C, self.F = to_dev(torch, A, B, C, F)
        N, M, R = F.shape
        self.R = R
        self.desc, self._keep = btd.make_desc(N, M, P, depth, R)
        self.fb, self.sb = btd.workspace_bytes(N, M, P, depth, R)
        self._fws, self.fptr = btd._aligned_buffer(self.fb, self.A.device)
        self._sws, self.sptr = btd._aligned_buffer(self.sb, self.A.device)
        self.X = torch.zeros_like(self.F)
        self.plans = []

    def enqueue(self, stream):
        sh = ctypes.c_void_p(stream.cuda_stream)
        h = ctypes.c_void_p()
        if self.fused:
            rc = self.L.btd_factor_solve(ctypes.byref(self.desc), self.A.data_ptr(), self.B.data_ptr(),
                                         self.C.data_ptr(), self.fptr, self.fb, self.R, self.F.data_ptr(),
                                         self.X.data_ptr(), self.sptr, self.sb, sh, ctypes.byref(h))
            assert rc == 0, rc
            self.plans.append(h)
            return h
        rc = self.L.btd_factor(ctypes.byref(self.desc), self.A.data_ptr(), self.B.data_ptr(), self.C.data_ptr(),
                               self.fptr, self.fb, sh, ctypes.byref(h))
        assert rc == 0, rc
        self.plans.append(h)
        rc = self.L.btd_solve(h, self.R, self.F.data_ptr(), self.X.data_ptr(), self.sptr, self.sb, sh)
        assert rc == 0, rc
        return h

    def release(self):
        self.torch.cuda.synchronize()
        for h in self.plans:
            self.L.btd_plan_destroy(h)
        self.plans = []


@pytest.mark.parametrize("N,M,R,P,depth,fused", [(80, 16, 2, 16, 1, False), (40, 33, 3, 6, 0, False),
                                                   (80, 16, 2, 16, 1, True), (200, 32, 3, 40, 2, True)])
def test_graph_replay_matches_eager(N, M, R, P, depth, fused):
    """fused: the graph holds one btd_factor_solve call (its right-hand-side
    side stream is part of the captured fork and join)."""
    torch = require_gpu()
    print(f"case graph N={N} M={M} R={R} P={P} depth={depth} fused={fused}", flush=True)
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=700 + N)
    A2, B2, C2, F2 = inputs.diag_dominant(N, M, R, seed=900 + N)
    run, other = AbiRun(torch, A, B, C, F, P, depth, fused), AbiRun(torch, A2, B2, C2, F2, P, depth)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h = run.enqueue(s)          # eager, also creates the library's side streams
    torch.cuda.synchronize()
    status = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert btd.lib().btd_get_info(h, *(ctypes.byref(v) for v in status)) == 0
    assert status[0].value == 0
    X_eager = run.X.cpu().numpy().copy()
    assert_parity(X_eager, oracle.dm_solve(A, B, C, F, P, depth=depth), 1e-10)
    run.release()

    g = torch.cuda.CUDAGraph()
    run.X.zero_()
    with torch.cuda.graph(g, stream=s):
        run.enqueue(s)
    torch.cuda.synchronize()
    for rep in range(3):
        run.X.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(run.X.cpu().numpy(), X_eager), f"replay {rep} differs from the eager solve"
        other.enqueue(torch.cuda.current_stream())   # eager work between the replays
        torch.cuda.synchronize()
        other.release()
    del g
    run.release()
