"""Serving loop over the solver: requests for solves of different sizes arrive
at random times; each is admitted as soon as a stream slot and enough of the
device-memory budget are free (continuous batching: requests that arrive while
others run are admitted as slots and memory free up, and their work overlaps
on the device), factored -- or served from a resident factorization, least
recently used ones evicted when the budget runs short -- solved, and checked
with the FP64 residual on its slot's stream.  The arithmetic is the library's
(btd_factor / btd_solve / btd_residual on the slot's stream); this module only
schedules, accounts for memory and measures latency.

Run as a module:
    python -m paper_1505_06864_amd.serve --mix full --rate 2000 --seconds 60
which prints one JSON line: offered and served rates, latency percentiles of
the served requests, the queue left at the end of the window, reuse hits,
evictions, peak bytes held, and the largest residual of any served result.
"""
import bisect
import collections
import ctypes
import json
import time

import numpy as np

from . import btd, inputs

DEPTH = 10
COUPLING_ROWS = 1
MAX_NRHS = 8


class System:
    """A block-tridiagonal system on the device and the plan settings it is
    factored with."""

    def __init__(self, name, A, B, C, P, max_nrhs, rhs_counts):
        self.name, self.A, self.B, self.C = name, A, B, C
        self.P, self.max_nrhs, self.rhs_counts = P, max_nrhs, tuple(rhs_counts)
        self.N, self.M = A.shape[0], A.shape[1]


class Request:
    """One solve: system `key` (a System), right-hand side F (a device
    tensor, or None: R columns drawn from N(0, 1) on the device with seed
    `seed` when the request is admitted)."""

    def __init__(self, rid, key, arrival, system, F=None, R=1, seed=0):
        self.rid, self.key, self.arrival = rid, key, arrival
        self.system = system
        self.F = F
        self.R = F.shape[2] if F is not None else R
        self.seed = seed
        self.X = None
        self.res = None               # device tensor of R relative residuals
        self.t_start = self.t_done = None
        self.factored = False


def footprint(sy, R):
    """Arena bytes of a system's factor workspace, and the blocks of one
    request with R columns: solve workspace, F, X, residual work and output
    (each rounded up to 256 bytes)."""
    if not hasattr(sy, "_bytes"):
        sy._bytes = btd.workspace_bytes(sy.N, sy.M, sy.P, DEPTH, sy.max_nrhs, None, COUPLING_ROWS)
    fbytes, sbytes = sy._bytes
    a = Arena.ALIGN
    up = lambda x: (int(x) + a - 1) // a * a
    parts = [up(sbytes), up(8 * sy.N * sy.M * R), up(8 * sy.N * sy.M * R),
             up(max(btd.lib().btd_residual_work_bytes(sy.N, sy.M, R), 8)), up(8 * R)]
    return up(fbytes), parts


class Arena:
    """First-fit sub-allocator over one device buffer of the budget's size
    (256-byte aligned blocks, neighbours merged on release).  The library
    takes plain workspace pointers, so every workspace of the server comes
    from here: the budget is exact, and no block is ever handed back to the
    device allocator while the loop runs."""

    ALIGN = 256

    def __init__(self, torch, nbytes, device):
        self.buf = torch.empty(int(nbytes) + self.ALIGN, dtype=torch.uint8, device=device)
        self.base = (self.buf.data_ptr() + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        self.size = int(nbytes) // self.ALIGN * self.ALIGN
        self.offs, self.lens = [0], [self.size]          # free blocks, sorted by offset

    def alloc(self, n):
        n = (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for k, ln in enumerate(self.lens):
            if ln >= n:
                off = self.offs[k]
                if ln == n:
                    del self.offs[k], self.lens[k]
                else:
                    self.offs[k] += n
                    self.lens[k] -= n
                return off, n
        return None

    def release(self, off, n):
        k = bisect.bisect_left(self.offs, off)
        self.offs.insert(k, off)
        self.lens.insert(k, n)
        if k + 1 < len(self.offs) and self.offs[k] + self.lens[k] == self.offs[k + 1]:
            self.lens[k] += self.lens.pop(k + 1)
            self.offs.pop(k + 1)
        if k > 0 and self.offs[k - 1] + self.lens[k - 1] == self.offs[k]:
            self.lens[k - 1] += self.lens.pop(k)
            self.offs.pop(k)

    def tensor(self, off, shape, torch):
        """A float64 tensor viewing arena bytes [off, off + 8 prod(shape))."""
        n = int(np.prod(shape))
        start = self.base - self.buf.data_ptr() + off
        return self.buf[start:start + 8 * n].view(torch.float64).view(*shape)


class Resident:
    """A factored system held in the arena (the library's plan handle)."""

    def __init__(self, handle, block):
        self.handle, self.block = handle, block


class Server:
    """Stream slots plus resident factorizations under a byte budget (the
    library's workspaces: factor workspace of each resident plan; solve
    workspace, right-hand side, solution and residual arrays of each running
    request), all carved from one arena of the budget's size."""

    def __init__(self, budget_bytes, slots=4, device="cuda", keep_results=False, check=True):
        import torch
        self.torch = torch
        self.keep = keep_results
        self.check = check
        self.budget = int(budget_bytes)
        self.arena = Arena(torch, self.budget, device)
        self.lib = btd.lib()
        self.streams = [torch.cuda.Stream(device) for _ in range(slots)]
        self.running = {}                                # slot -> (request, event, bytes)
        self.resident = collections.OrderedDict()        # key -> [plan, bytes, running solves, factored event]
        self.used = 0
        self.peak = 0
        self.evictions = 0

    def _sizes(self, req):
        return footprint(req.system, req.R)

    def _need(self, req):
        fbytes, parts = self._sizes(req)
        return (0 if req.key in self.resident else fbytes), sum(parts)

    def _make_room(self, need, keep=None):
        """Evict idle resident factorizations, least recently used first, until
        `need` more bytes fit; `keep` (the system the request reuses) is never
        evicted."""
        while self.used + need > self.budget:
            victim = next((k for k, v in self.resident.items() if v[2] == 0 and k != keep), None)
            if victim is None:
                return False
            res, nbytes = self.resident.pop(victim)[:2]
            # no solve of this plan is running and its factorisation finished
            # before its last solve did: its workspace is free to reuse
            self.lib.btd_plan_destroy(res.handle)
            self.arena.release(*res.block)
            self.used -= nbytes
            self.evictions += 1
        return True

    def _alloc(self, fneed, rneed, keep):
        """Arena blocks for a factor workspace (fneed > 0) and the request's
        own arrays, evicting idle factorizations (least recently used first,
        never `keep`) until both fit; None when they cannot."""
        while True:
            fb = self.arena.alloc(fneed) if fneed else (0, 0)
            rb = self.arena.alloc(rneed) if fb is not None else None
            if fb is not None and rb is not None:
                return fb, rb
            if fb is not None and fneed:
                self.arena.release(*fb)
            victim = next((k for k, v in self.resident.items() if v[2] == 0 and k != keep), None)
            if victim is None:
                return None
            res, nbytes = self.resident.pop(victim)[:2]
            self.lib.btd_plan_destroy(res.handle)
            self.arena.release(*res.block)
            self.used -= nbytes
            self.evictions += 1

    def try_launch(self, req, now):
        slot = next((s for s in range(len(self.streams)) if s not in self.running), None)
        if slot is None:
            return False
        fneed, rneed = self._need(req)
        if fneed + rneed > self.budget or not self._make_room(fneed + rneed, keep=req.key):
            return False
        blocks = self._alloc(fneed, rneed, req.key)   # the byte count fits; the arena may still be fragmented
        if blocks is None:
            return False
        fb, rb = blocks
        s = self.streams[slot]
        torch, L = self.torch, self.lib
        sy = req.system
        sh = ctypes.c_void_p(s.cuda_stream)
        if req.key in self.resident:
            entry = self.resident[req.key]
            self.resident.move_to_end(req.key)
            s.wait_event(entry[3])   # its factorisation may still run on another slot
        else:
            desc, _keep = btd.make_desc(sy.N, sy.M, sy.P, DEPTH, sy.max_nrhs, None, COUPLING_ROWS)
            h = ctypes.c_void_p()
            rc = L.btd_factor(ctypes.byref(desc), sy.A.data_ptr(), sy.B.data_ptr(), sy.C.data_ptr(),
                              self.arena.base + fb[0], fb[1], sh, ctypes.byref(h))
            if rc != btd.BTD_OK:
                raise btd.BtdError(rc, "btd_factor")
            factored = torch.cuda.Event()
            factored.record(s)
            entry = self.resident[req.key] = [Resident(h, fb), fb[1], 0, factored]
            self.used += fb[1]
            req.factored = True
        entry[2] += 1
        _, parts = self._sizes(req)
        offs = np.cumsum([rb[0]] + parts[:-1])
        sws, fo, xo, wo, oo = (int(o) for o in offs)
        shape = (sy.N, sy.M, req.R)
        with torch.cuda.stream(s):
            F = self.arena.tensor(fo, shape, torch)
            if req.F is None:
                g = torch.Generator(device=sy.A.device)
                g.manual_seed(req.seed)
                F.normal_(generator=g)
            else:
                F.copy_(req.F)
            X = self.arena.tensor(xo, shape, torch)
        rc = L.btd_solve(entry[0].handle, req.R, F.data_ptr(), X.data_ptr(), self.arena.base + sws, parts[0], sh)
        if rc != btd.BTD_OK:
            raise btd.BtdError(rc, "btd_solve")
        out = self.arena.tensor(oo, (req.R,), torch)
        if self.check:
            rc = L.btd_residual(sy.N, sy.M, req.R, sy.A.data_ptr(), sy.B.data_ptr(), sy.C.data_ptr(), X.data_ptr(),
                                F.data_ptr(), out.data_ptr(), self.arena.base + wo, sh)
            if rc != btd.BTD_OK:
                raise btd.BtdError(rc, "btd_residual")
        ev = torch.cuda.Event()
        ev.record(s)
        req.F, req.X, req.res = F, X, (out if self.check else None)
        self.used += rb[1]
        assert self.used <= self.budget, (self.used, self.budget)
        self.peak = max(self.peak, self.used)
        req.t_start = now
        self.running[slot] = (req, ev, rb)
        return True

    def poll(self, now):
        done = []
        for slot, (req, ev, rb) in list(self.running.items()):
            if ev.query():
                req.t_done = now
                self.resident[req.key][2] -= 1
                if req.res is not None:
                    req.res = float(req.res.max().item())
                if self.keep:     # results outlive the arena block
                    req.F, req.X = req.F.clone(), req.X.clone()
                else:
                    req.X = req.F = None
                self.arena.release(*rb)
                self.used -= rb[1]
                del self.running[slot]
                done.append(req)
        return done

    def close(self):
        self.torch.cuda.synchronize()
        for entry in self.resident.values():
            self.lib.btd_plan_destroy(entry[0].handle)
            self.arena.release(*entry[0].block)
        self.resident.clear()
        self.used = 0


def serve(requests, budget_bytes, slots=4, keep_results=False, window=None, check=True):
    """Run the requests (sorted by arrival time, seconds from now) through a
    Server.  With `window` (seconds) arrivals after it are not admitted, the
    requests still waiting at its end are left unserved (counted in
    `queue_at_end`) and the running ones finish.  Returns the completed
    requests and the server's counters."""
    srv = Server(budget_bytes, slots, keep_results=keep_results, check=check)
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting = collections.deque()
    finished = []
    max_queue = 0
    t0 = time.perf_counter()
    while pending or waiting or srv.running:
        now = time.perf_counter() - t0
        if window is not None and now > window:
            if not srv.running:
                break
            finished.extend(srv.poll(now))
            continue
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        max_queue = max(max_queue, len(waiting))
        finished.extend(srv.poll(now))
        while waiting and srv.try_launch(waiting[0], now):
            waiting.popleft()
        if not srv.running and waiting:
            raise RuntimeError(f"request {waiting[0].rid} does not fit the budget")
    counters = {"evictions": srv.evictions, "peak_bytes": srv.peak,
                "factored": sum(r.factored for r in finished),
                "reused": sum(not r.factored for r in finished),
                "queue_at_end": len(waiting) + len(pending) if window is not None else 0,
                "max_queue": max_queue}
    srv.close()
    return finished, counters


def small_pool(torch, sizes, device="cuda", max_nrhs=MAX_NRHS):
    """Systems of the given (N, M) sizes (diagonally dominant blocks)."""
    pool = []
    for q, (N, M) in enumerate(sizes):
        A, B, C, _ = inputs.diag_dominant(N, M, 1, seed=4000 + q)
        P = max(1, min(64, (N + 1) // 8))
        pool.append(System(f"N{N}M{M}", *(torch.from_numpy(a).to(device) for a in (A, B, C)), P, max_nrhs, (1, 8)))
    return pool


def full_pool(torch, device="cuda", uneven=16, seed=4):
    """The serving mix's systems by family: the Faddeev-type workload
    (N=2048, M=128, R=4), the large workload (N=4096, M=256, R in {1, 64}),
    and batched uneven systems (N ~ U{32..1024}, M in {32, 64, 128, 192},
    R in {1, 8, 32}, per-system seeds)."""
    rng = np.random.default_rng(seed)
    fam = {"faddeev": [], "large": [], "uneven": []}
    A, B, C, _ = inputs.cfg_faddeev()
    fam["faddeev"].append(System("faddeev", *(torch.from_numpy(a).to(device) for a in (A, B, C)), 256, 4, (4,)))
    A, B, C, _ = inputs.cfg_large(R=1)
    fam["large"].append(System("large", *(torch.from_numpy(a).to(device) for a in (A, B, C)), 256, 64, (1, 64)))
    del A, B, C
    for s in range(uneven):
        N = int(rng.integers(32, 1025))
        M = int(rng.choice([32, 64, 128, 192]))
        A, B, C, _ = inputs.diag_dominant(N, M, 1, seed=3000 + s)
        P = max(1, min(256, (N + 1) // 8))
        fam["uneven"].append(System(f"uneven{s}", *(torch.from_numpy(a).to(device) for a in (A, B, C)), P, 32,
                                    (1, 8, 32)))
    return fam


def make_load(torch, rate, seconds, seed=4, reuse=0.3, sizes=None, device="cuda", recent=8, pool=None,
              weights=None):
    """Poisson arrivals at `rate` per second for `seconds`; a request reuses
    one of the `recent` latest systems (new right-hand side) with probability
    `reuse`, else it brings a new system (a new factorization), drawn from
    the pool (a list of Systems, or a dict family -> list drawn by `weights`).
    Each request's right-hand side is drawn on the device when it is admitted."""
    rng = np.random.default_rng(seed)
    if pool is None:
        pool = small_pool(torch, sizes or [(64, 32), (128, 32), (256, 64), (512, 64), (256, 128), (1024, 128),
                                           (512, 256)], device)
    if isinstance(pool, dict):
        names = sorted(pool)
        w = np.array([(weights or {}).get(n, 1.0) for n in names], dtype=float)
        w /= w.sum()
    reqs, t, keys, sys_of = [], 0.0, [], {}
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        if keys and rng.random() < reuse:
            key = keys[-1 - rng.integers(min(recent, len(keys)))]
            system = sys_of[key]
        else:
            key = len(keys)
            keys.append(key)
            if isinstance(pool, dict):
                fam = pool[names[rng.choice(len(names), p=w)]]
                system = fam[rng.integers(len(fam))]
            else:
                system = pool[rng.integers(len(pool))]
            sys_of[key] = system
        R = int(rng.choice(system.rhs_counts))
        reqs.append(Request(len(reqs), key, t, system, None, R=R, seed=seed * 1000003 + len(reqs)))
    return reqs


def stats(finished, counters, window=None):
    lat = np.array([r.t_done - r.arrival for r in finished]) * 1e3
    span = window if window is not None else max(r.t_done for r in finished) - min(r.arrival for r in finished)
    res = [r.res for r in finished if r.res is not None]
    return {"served": len(finished), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "served_per_s": len(finished) / max(span, 1e-9),
            "residual_max": max(res) if res else None, **counters}


def main():
    import argparse
    import os

    # one stream per request: the plans do not split their subsystems over
    # the library's shared side streams, so requests overlap freely
    os.environ.setdefault("BTD_STREAM_GROUPS", "1")
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--mix", choices=("small", "full"), default="full",
                    help="full: the Faddeev-type, large and uneven systems; small: sizes up to N=1024, M=256")
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--reuse", type=float, default=0.3)
    args = ap.parse_args()
    budget = args.budget_gib * 2**30
    pool = full_pool(torch) if args.mix == "full" else None
    warm = make_load(torch, 20, 0.5, seed=1, pool=pool)
    serve(warm, budget, args.slots)
    reqs = make_load(torch, args.rate, args.seconds, reuse=args.reuse, pool=pool)
    t0 = time.perf_counter()
    finished, counters = serve(reqs, budget, args.slots, window=args.seconds)
    wall = time.perf_counter() - t0
    out = stats(finished, counters, window=args.seconds)
    by = collections.Counter(r.system.name if args.mix == "small" else r.system.name.rstrip("0123456789")
                             for r in finished)
    out.update({"mix": args.mix, "offered": len(reqs), "offered_per_s": len(reqs) / args.seconds,
                "seconds": args.seconds, "wall_s": wall, "slots": args.slots, "budget_gib": args.budget_gib,
                "reuse": args.reuse, "served_by_family": dict(by)})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
