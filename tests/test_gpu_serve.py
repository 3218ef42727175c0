"""GPU: the serving loop.  Requests of different sizes arrive while others
run on the device; each is admitted when a stream slot and the memory budget
allow (evicting idle resident factorizations), and reuses a resident
factorization when its system is still there.  Every result must equal, bit
for bit, the same solve run alone (the kernels fix their reduction orders),
match the FP64 oracle and meet the residual bar; the budget is never
exceeded.
"""
import pytest

import oracle
from paper_1505_06864_amd import btd, serve
from gpu_util import assert_parity, require_gpu

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
    assert counters["peak_bytes"] <= budget
    refs = {}
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
        # the FP64 oracle on the same system and right-hand side
        if r.key not in refs:
            refs[r.key] = tuple(t.cpu().numpy() for t in (A, B, C))
        Ah, Bh, Ch = refs[r.key]
        Fh = r.F.cpu().numpy()
        assert_parity(r.X.cpu().numpy(), oracle.dm_solve(Ah, Bh, Ch, Fh, P, depth=1), 1e-10)


def test_reused_system_is_never_evicted_for_itself():
    """A request that reuses a resident factorization while the budget is
    short must not evict that very factorization (and factor it again past
    the budget); other idle factorizations go, least recently used first.
    Two systems, room for both factorizations and one and a half solves,
    two slots, all requests at once (keys 0, 1, 0, 0, 1, 0):
      r0 factors system 0; r1 waits for room, then factors system 1;
      r2 (reuse of 0) waits while r1 runs: system 0 is idle but is the one
      it reuses; r3 (reuse of 0) finds system 1 idle and evicts it;
      r4 factors system 1 again once both reuses are done; r5 reuses 0.
    So 3 factorizations, 3 reuses, 1 eviction, and the budget holds."""
    import numpy as np
    torch = require_gpu()
    N, M = 64, 32
    P = max(1, min(64, (N + 1) // 8))
    systems = []
    for q in range(2):
        A, B, C, _ = serve.inputs.diag_dominant(N, M, 1, seed=4100 + q)
        systems.append(tuple(torch.from_numpy(a).cuda() for a in (A, B, C)) + (P,))
    rng = np.random.default_rng(3)
    keys = [0, 1, 0, 0, 1, 0]
    reqs = [serve.Request(i, k, 0.0, systems[k], torch.from_numpy(rng.standard_normal((N, M, 1))).cuda())
            for i, k in enumerate(keys)]
    f, sb = btd.workspace_bytes(N, M, P, serve.DEPTH, serve.MAX_NRHS, None, serve.COUPLING_ROWS)
    budget = 2 * f + sb + sb // 2
    finished, counters = serve.serve(reqs, budget, slots=2, keep_results=True)
    assert len(finished) == len(reqs)
    assert (counters["factored"], counters["reused"], counters["evictions"]) == (3, 3, 1), counters
    assert counters["peak_bytes"] <= budget
