"""Serving loop over the solver: requests for solves of different sizes arrive
at random times; each is admitted as soon as a stream slot and enough of the
device-memory budget are free, factored (or served from a resident
factorization, least recently used ones evicted when the budget runs short)
and solved on its slot's stream while other requests run.  The arithmetic is
the library's (btd_factor / btd_solve on the slot's stream); this module only
schedules, accounts for memory and measures latency.

Run as a module for a synthetic load:
    python -m paper_1505_06864_amd.serve --rate 200 --seconds 5
which prints one JSON line (latency percentiles, offered and served rates,
reuse hits, evictions).
"""
import collections
import json
import time

import numpy as np

from . import btd, inputs

DEPTH = 10
COUPLING_ROWS = 1
MAX_NRHS = 8


class Request:
    """One solve: system `key` (A, B, C on the device), right-hand side F."""

    def __init__(self, rid, key, arrival, system, F):
        self.rid, self.key, self.arrival = rid, key, arrival
        self.system = system          # (A, B, C, P) device tensors and subsystem count
        self.F = F
        self.X = None
        self.t_start = self.t_done = None
        self.factored = False


class Server:
    """Stream slots plus resident factorizations under a byte budget (the
    library's workspaces: factor workspace of each resident plan, solve
    workspace of each running solve)."""

    def __init__(self, budget_bytes, slots=4, device="cuda", keep_results=False):
        import torch
        self.torch = torch
        self.keep = keep_results
        self.budget = int(budget_bytes)
        self.streams = [torch.cuda.Stream(device) for _ in range(slots)]
        self.running = {}                                # slot -> (request, event, solve bytes)
        self.resident = collections.OrderedDict()        # key -> [plan, bytes, running solves, factored event]
        self.used = 0
        self.peak = 0
        self.evictions = 0

    def _need(self, req):
        A, _, _, P = req.system
        N, M = A.shape[0], A.shape[1]
        fbytes, sbytes = btd.workspace_bytes(N, M, P, DEPTH, MAX_NRHS, None, COUPLING_ROWS)
        return (0 if req.key in self.resident else fbytes), sbytes

    def _make_room(self, need, keep=None):
        """Evict idle resident factorizations, least recently used first, until
        `need` more bytes fit; `keep` (the system the request reuses) is never
        evicted."""
        while self.used + need > self.budget:
            victim = next((k for k, v in self.resident.items() if v[2] == 0 and k != keep), None)
            if victim is None:
                return False
            plan, nbytes = self.resident.pop(victim)[:2]
            # no solve of this plan is running and its factorisation finished
            # before its last solve did: release it without a device-wide wait
            plan.release_after_work()
            self.used -= nbytes
            self.evictions += 1
        return True

    def try_launch(self, req, now):
        slot = next((s for s in range(len(self.streams)) if s not in self.running), None)
        if slot is None:
            return False
        fneed, sneed = self._need(req)
        if fneed + sneed > self.budget or not self._make_room(fneed + sneed, keep=req.key):
            return False
        s = self.streams[slot]
        torch = self.torch
        with torch.cuda.stream(s):
            if req.key in self.resident:
                entry = self.resident[req.key]
                self.resident.move_to_end(req.key)
                s.wait_event(entry[3])   # its factorisation may still run on another slot
            else:
                A, B, C, P = req.system
                plan = btd.factor(A, B, C, P=P, depth=DEPTH, max_nrhs=MAX_NRHS, stream=s,
                                  coupling_rows=COUPLING_ROWS)
                factored = torch.cuda.Event()
                factored.record(s)
                entry = self.resident[req.key] = [plan, plan.factor_bytes, 0, factored]
                self.used += plan.factor_bytes
                req.factored = True
            entry[2] += 1
            req.X = entry[0].solve(req.F, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.used += sneed
        assert self.used <= self.budget, (self.used, self.budget)
        self.peak = max(self.peak, self.used)
        req.t_start = now
        self.running[slot] = (req, ev, sneed)
        return True

    def poll(self, now):
        done = []
        for slot, (req, ev, sneed) in list(self.running.items()):
            if ev.query():
                req.t_done = now
                self.resident[req.key][2] -= 1
                self.used -= sneed
                del self.running[slot]
                if not self.keep:
                    req.X = req.F = None
                done.append(req)
        return done

    def close(self):
        self.torch.cuda.synchronize()
        for entry in self.resident.values():
            entry[0].destroy()
        self.resident.clear()
        self.used = 0


def serve(requests, budget_bytes, slots=4, keep_results=False):
    """Run the requests (sorted by arrival time, seconds from now) through a
    Server; returns the completed requests and the server's counters."""
    srv = Server(budget_bytes, slots, keep_results=keep_results)
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting = collections.deque()
    finished = []
    t0 = time.perf_counter()
    while pending or waiting or srv.running:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        finished.extend(srv.poll(now))
        while waiting and srv.try_launch(waiting[0], now):
            waiting.popleft()
        if not srv.running and waiting:
            raise RuntimeError(f"request {waiting[0].rid} does not fit the budget")
    counters = {"evictions": srv.evictions, "peak_bytes": srv.peak,
                "factored": sum(r.factored for r in finished),
                "reused": sum(not r.factored for r in finished)}
    srv.close()
    return finished, counters


def make_load(torch, rate, seconds, seed=4, reuse=0.3, sizes=None, device="cuda", recent=8):
    """Poisson arrivals at `rate` per second for `seconds`; a request reuses
    one of the `recent` latest systems (new right-hand side) with probability
    `reuse`, else it brings a new one, drawn from a pool of systems generated
    beforehand on the device."""
    rng = np.random.default_rng(seed)
    sizes = sizes or [(64, 32), (128, 32), (256, 64), (512, 64), (256, 128), (1024, 128), (512, 256)]
    pool = []
    for q, (N, M) in enumerate(sizes):
        A, B, C, _ = inputs.diag_dominant(N, M, 1, seed=4000 + q)
        P = max(1, min(64, (N + 1) // 8))
        pool.append(tuple(torch.from_numpy(a).to(device) for a in (A, B, C)) + (P,))
    reqs, t, keys = [], 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        if keys and rng.random() < reuse:
            key = keys[-1 - rng.integers(min(recent, len(keys)))]
            system = next(r.system for r in reqs if r.key == key)
        else:
            key = len(keys)
            keys.append(key)
            system = pool[rng.integers(len(pool))]
        A = system[0]
        R = int(rng.choice([1, 8]))
        F = torch.from_numpy(rng.standard_normal((A.shape[0], A.shape[1], R))).to(device)
        reqs.append(Request(len(reqs), key, t, system, F))
    return reqs


def stats(finished, counters):
    lat = np.array([r.t_done - r.arrival for r in finished]) * 1e3
    span = max(r.t_done for r in finished) - min(r.arrival for r in finished)
    last = max(r.arrival for r in finished)
    return {"requests": len(finished), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "offered_per_s": len(finished) / max(last, 1e-9),
            "served_per_s": len(finished) / max(span, 1e-9), **counters}


def main():
    import argparse
    import os

    # one stream per request: the plans do not split their subsystems over
    # the library's shared side streams, so requests overlap freely
    os.environ.setdefault("BTD_STREAM_GROUPS", "1")
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--seconds", type=float, default=5.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    args = ap.parse_args()
    warm = make_load(torch, 50, 0.2, seed=1)
    serve(warm, args.budget_gib * 2**30, args.slots)
    reqs = make_load(torch, args.rate, args.seconds)
    finished, counters = serve(reqs, args.budget_gib * 2**30, args.slots)
    out = stats(finished, counters)
    out.update({"rate": args.rate, "seconds": args.seconds, "slots": args.slots, "budget_gib": args.budget_gib})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
