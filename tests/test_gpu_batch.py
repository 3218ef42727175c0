"""GPU: batched uneven systems.  Systems of one block size stacked into one
block-tridiagonal system with zero junction blocks and solved by one plan:
every system's solution against the FP64 oracle solving that system alone
(FP64 and FP32 products with refinement), the autotuner's choice valid and
cached, and a graph replay of the whole batch equal to the eager run.
"""
import numpy as np
import pytest

import oracle
from paper_1505_06864_amd import batch, inputs
from gpu_util import assert_parity, require_gpu

pytestmark = pytest.mark.gpu


def make_groups(torch, count=36, seed=5):
    specs = inputs.uneven_specs(count, seed=seed, n_range=(8, 120), blocks=(8, 16, 40, 64), rhs=(1, 4, 9))
    systems = [inputs.uneven_system(sp, s) for s, sp in enumerate(specs)]
    groups = []
    for M, idx in sorted(batch.group_by_block_size(specs).items()):
        g = batch.Group.stack([systems[s][:3] for s in idx], [specs[s][2] for s in idx])
        g.systems = idx
        F = g.stack_rhs([systems[s][3] for s in idx])
        groups.append((g, F))
    return specs, systems, groups


@pytest.mark.parametrize("prec,fused", [("f64", False), ("f64", True), ("f32_refine", False)])
def test_batched_systems_match_oracle(prec, fused):
    torch = require_gpu()
    specs, systems, groups = make_groups(torch)
    tuner = batch.Tuner(fused=fused)
    for g, F in groups:
        P, depth, crow = tuner.choose(g, F, prec)
        print(f"group M={g.M} systems={len(g.rows)} rows={g.N} R={g.R} -> P={P} depth={depth} "
              f"coupling_rows={crow}", flush=True)
        assert 1 <= P <= (g.N + 1) // 2
        assert tuner.choose(g, F, prec) == (P, depth, crow)       # cached
        run = batch.GroupRun(g, P, depth, crow, prec, fused=fused)
        X = run.step(F)
        assert run.info() == (0, -1, -1)
        for s, x in zip(g.systems, g.split(X)):
            A, B, C, Fs = systems[s]
            N = A.shape[0]
            Ps = max(1, min(4, (N + 1) // 4))
            assert_parity(x.cpu().numpy(), oracle.dm_solve(A, B, C, Fs, Ps, depth=0), 1e-10)
        if prec == "f32_refine":
            assert max(run.res) <= 1e-12
        run.release()


@pytest.mark.parametrize("fused", [False, True])
def test_batched_graph_replay_matches_eager(fused):
    torch = require_gpu()
    specs, systems, groups = make_groups(torch, count=20, seed=6)
    fmax = smax = 0
    from paper_1505_06864_amd import btd
    params = [(max(1, (g.N + 1) // 9), 10, 1) for g, _ in groups]
    for (g, _), (P, d, c) in zip(groups, params):
        f, s = btd.workspace_bytes(g.N, g.M, P, d, g.R, None, c)
        fmax, smax = max(fmax, f), max(smax, s)
    shared = (torch.empty(fmax + 256, dtype=torch.uint8, device="cuda"),
              torch.empty(smax + 256, dtype=torch.uint8, device="cuda"))
    runs = [batch.GroupRun(g, P, d, c, "f64", shared=shared, fused=fused) for (g, _), (P, d, c) in zip(groups, params)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for run in runs:
        run.use_stream(s)
    with torch.cuda.stream(s):
        for run, (g, F) in zip(runs, groups):
            run.step(F)
    torch.cuda.synchronize()
    eager = [run.X.clone() for run in runs]
    for run in runs:
        run.release()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        for run, (g, F) in zip(runs, groups):
            run.step(F)
    for rep in range(3):
        for run in runs:
            run.X.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for run, x in zip(runs, eager):
            assert torch.equal(run.X, x), f"replay {rep}"
    del graph
    for run in runs:
        run.release()
    for (g, _), x in zip(groups, eager):
        for sidx, xs in zip(g.systems, g.split(x)):
            A, B, C, Fs = systems[sidx]
            assert_parity(xs.cpu().numpy(), oracle.dm_solve(A, B, C, Fs, 1), 1e-10)
