"""GPU: the serving loop.  Requests of different sizes arrive while others
run on the device; each is admitted when a stream slot and the memory budget
allow (evicting idle resident factorizations), and reuses a resident
factorization when its system is still there.  Every result must equal, bit
for bit, the same solve run alone (the kernels fix their reduction orders),
and meet the residual bar.
"""
import pytest

from paper_1505_06864_amd import btd, serve
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_the_mix():
    torch = require_gpu()
    sizes = [(40, 16), (64, 32), (100, 24), (33, 8)]
    reqs = serve.make_load(torch, rate=600.0, seconds=0.08, seed=7, sizes=sizes)
    assert len(reqs) >= 20
    fmax = max(btd.workspace_bytes(N, M, max(1, min(64, (N + 1) // 8)), serve.DEPTH, serve.MAX_NRHS, None,
                                   serve.COUPLING_ROWS)[0] for N, M in sizes)
    smax = max(btd.workspace_bytes(N, M, max(1, min(64, (N + 1) // 8)), serve.DEPTH, serve.MAX_NRHS, None,
                                   serve.COUPLING_ROWS)[1] for N, M in sizes)
    budget = 2 * fmax + 3 * smax          # room for about two resident factorizations
    print(f"serve {len(reqs)} requests, budget {budget} bytes", flush=True)
    finished, counters = serve.serve(reqs, budget, slots=3, keep_results=True)
    assert len(finished) == len(reqs)
    assert counters["evictions"] > 0 and counters["reused"] > 0, counters
    for r in finished:
        A, B, C, P = r.system
        plan = btd.factor(A, B, C, P=P, depth=serve.DEPTH, max_nrhs=serve.MAX_NRHS,
                          coupling_rows=serve.COUPLING_ROWS)
        X = plan.solve(r.F)
        assert plan.info() == (0, -1, -1)
        assert torch.equal(X, r.X), f"request {r.rid} differs from the same solve alone"
        res = btd.residual(A, B, C, X, r.F).max().item()
        assert res <= 1e-12, (r.rid, res)
        plan.destroy()
