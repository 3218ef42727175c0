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
    pool = {r.system.name: r.system for r in reqs}
    fmax = max(serve.footprint(sy, serve.MAX_NRHS)[0] for sy in pool.values())
    smax = max(sum(serve.footprint(sy, serve.MAX_NRHS)[1]) for sy in pool.values())
    budget = 2 * fmax + 3 * smax          # room for about two resident factorizations
    print(f"serve {len(reqs)} requests, budget {budget} bytes", flush=True)
    finished, counters = serve.serve(reqs, budget, slots=3, keep_results=True)
    assert len(finished) == len(reqs)
    assert counters["evictions"] > 0 and counters["reused"] > 0, counters
    assert counters["peak_bytes"] <= budget
    refs = {}
    for r in finished:
        sy = r.system
        A, B, C, P = sy.A, sy.B, sy.C, sy.P
        assert r.res is not None and r.res <= 1e-12, (r.rid, r.res)
        plan = btd.factor(A, B, C, P=P, depth=serve.DEPTH, max_nrhs=sy.max_nrhs,
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
        systems.append(serve.System(f"s{q}", *(torch.from_numpy(a).cuda() for a in (A, B, C)), P, serve.MAX_NRHS,
                                    (1,)))
    rng = np.random.default_rng(3)
    keys = [0, 1, 0, 0, 1, 0]
    reqs = [serve.Request(i, k, 0.0, systems[k], torch.from_numpy(rng.standard_normal((N, M, 1))).cuda())
            for i, k in enumerate(keys)]
    f, parts = serve.footprint(systems[0], 1)
    sb = sum(parts)                       # one request's own arrays
    budget = 2 * f + sb + sb // 2
    finished, counters = serve.serve(reqs, budget, slots=2, keep_results=True)
    assert len(finished) == len(reqs)
    assert (counters["factored"], counters["reused"], counters["evictions"]) == (3, 3, 1), counters
    assert counters["peak_bytes"] <= budget


def test_serving_mix_families_match_oracle():
    """The serving mix's three families at reduced sizes (Faddeev-type
    banded blocks; dense blocks with shift 1.5 and 1 or 64 right-hand sides;
    uneven systems with M in {32, 64, 128, 192} and 1, 8 or 32 right-hand
    sides), arriving faster than they are served, 30% of them reusing a
    resident factorization: every result against the FP64 oracle."""
    import numpy as np
    torch = require_gpu()
    rng = np.random.default_rng(21)
    dev = "cuda"

    def system(name, arrays, P, max_nrhs, counts):
        return serve.System(name, *(torch.from_numpy(a).to(dev) for a in arrays[:3]), P, max_nrhs, counts)

    pool = {"faddeev": [system("faddeev", serve.inputs.faddeev_like(256, 128, 1, seed=22), 32, 4, (4,))],
            "large": [system("large", serve.inputs.diag_dominant(240, 256, 1, seed=23, shift=1.5), 32, 64, (1, 64))],
            "uneven": []}
    for q in range(5):
        N, M = int(rng.integers(32, 300)), int(rng.choice([32, 64, 128, 192]))
        pool["uneven"].append(system(f"uneven{q}", serve.inputs.diag_dominant(N, M, 1, seed=3100 + q),
                                     max(1, min(256, (N + 1) // 8)), 32, (1, 8, 32)))
    reqs = serve.make_load(torch, rate=300.0, seconds=0.12, seed=24, pool=pool)
    assert len(reqs) >= 15
    print(f"serve mix: {len(reqs)} requests", flush=True)
    finished, counters = serve.serve(reqs, 64 * 2**30, slots=4, keep_results=True)
    assert len(finished) == len(reqs) and counters["reused"] > 0, counters
    host = {}
    for r in finished:
        sy = r.system
        if sy.name not in host:
            host[sy.name] = tuple(t.cpu().numpy() for t in (sy.A, sy.B, sy.C))
        A, B, C = host[sy.name]
        F = r.F.cpu().numpy()
        assert r.res <= 1e-12, (r.rid, sy.name, r.res)
        assert_parity(r.X.cpu().numpy(), oracle.dm_solve(A, B, C, F, min(sy.P, 16), depth=1), 1e-10)
