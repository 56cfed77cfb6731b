"""Continuous batching of independent Helmholtz factor + solve requests.

A request is a model m on a grid, one or more frequencies and a block of
right-hand sides (point sources by default).  The server keeps a FIFO queue;
each scheduler iteration admits every queued request that fits, in arrival
order, until the chain limit of one batched launch sequence (16 chains; one
chain per frequency) or the HBM budget is reached.  Admitted requests are
factored together (one set of launches for all their chains) and solved
together, so requests that arrive while a batch runs join the next one.
By default the next batch is admitted and factored while the current one is
solved (two batches in flight, on two streams); its memory then counts
against the budget together with the batch in flight.  With lanes = L > 1
(`run_lanes`), L host threads each admit a batch, factor it and solve it on
a stream of their own, so batches on different grids run side by side and
a lane that finishes admits the next batch at once; the memory of every
batch in flight counts against the budget.
This is the paper's observation that the solves for different models are
independent (Appendix, "Parallelisation"), applied to a request stream.

Memory: a request needs its factors (helm_factor_bytes per frequency) plus
its solutions and refinement buffers (48 bytes per unknown and right-hand
side per frequency).  With `resident=True`, factors of requests that name a
`model_key` stay in HBM after the request completes, and are reused by later
requests with the same key, frequency and precision.  Resident factors count
against the budget and are evicted least-recently-used when room is needed.
A request larger than the whole budget is rejected.

    python -m paper_2301_10762_amd.serving --requests 32 --rate 200
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import math
import sys
import threading
import time

from .helm import pooled_stream

MAX_CHAINS = 16
BYTES_PER_UNKNOWN_RHS = 48


@dataclasses.dataclass
class ServeRequest:
    rid: int
    grid: object                 # helm.Grid
    m: object                    # FP64 model, length N (device tensor or array)
    omegas: list
    sources: list = None         # node indices of unit point sources ...
    B: object = None             # ... or an explicit [S][N] complex128 device block
    arrival: float = 0.0         # seconds, relative to the stream start
    model_key: object = None     # for resident factors
    precision: str = None        # "fp64" or "fp32_ir"; None: the backend's

    @property
    def S(self) -> int:
        return len(self.sources) if self.B is None else int(self.B.shape[0])


@dataclasses.dataclass
class ServeResult:
    rid: int
    X: list                      # per frequency, [S][N] complex128 device tensors
    infos: list
    arrival: float
    start: float
    done: float
    batch: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class _Prepared:
    batch: list
    t0: float
    Fs: dict = dataclasses.field(default_factory=dict)      # (request, frequency) -> factor
    slots: list = dataclasses.field(default_factory=list)   # entries of Fs to factor
    grids: list = dataclasses.field(default_factory=list)
    ms: list = dataclasses.field(default_factory=list)
    oms: list = dataclasses.field(default_factory=list)
    keys: set = dataclasses.field(default_factory=set)      # resident factors used
    precision: str = None                                    # of every request of the batch
    bytes: int = 0
    Bs: dict = None
    be: object = None                                        # backend (lane) that runs the batch


class HelmBackend:
    """The device path: helm.factor_batch / helm.solve_batch.  Factors are
    made on one stream and solved on another, so that a pipelined server
    can factor the next batch while the current one is solved."""

    def __init__(self, precision="fp32_ir", tol=1e-10, stream=None, solve_stream=None):
        from . import helm
        self.helm = helm
        self.precision = precision
        self.tol = tol
        self.stream = stream
        self.solve_stream = solve_stream if solve_stream is not None else stream
        self.factorisations = 0
        self.own = None          # a lane's stream: sync() waits for it alone

    def lane(self, k: int = 0):
        """A backend for lane k of run_lanes: factors, solves and its
        right-hand sides on a stream of its own, and sync() waiting for that
        stream only (a device-wide synchronisation would make a lane wait for
        the others' batches).  Lane k of every run uses the same pooled
        stream (pooled_stream), so memory freed by one run serves the next;
        two runs at once in one process share their lanes' streams, which
        orders their work but does not change results."""
        s = pooled_stream(("lane", k))
        b = HelmBackend(self.precision, self.tol, stream=s, solve_stream=s)
        b.own = s
        return b

    def stream_context(self):
        """Context in which the lane's tensors are made on its stream."""
        import contextlib
        import torch
        return torch.cuda.stream(self.own) if self.own is not None else contextlib.nullcontext()

    def factor_bytes(self, grid, precision=None) -> int:
        return self.helm.factor_bytes(grid, precision or self.precision)

    def factor(self, grids, ms, omegas, precision=None):
        self.factorisations += len(grids)
        return self.helm.factor_batch(grids, ms, omegas, precision or self.precision, self.stream)

    def rhs(self, req: ServeRequest):
        if req.B is not None:
            return req.B
        import torch
        B = torch.zeros((len(req.sources), req.grid.N), dtype=torch.complex128, device="cuda")
        idx = torch.as_tensor(list(req.sources), dtype=torch.int64, device="cuda")
        B[torch.arange(len(req.sources), device="cuda"), idx] = 1.0
        return B

    def model(self, req: ServeRequest):
        import torch
        if isinstance(req.m, torch.Tensor) and req.m.is_cuda:
            return req.m
        return torch.as_tensor(req.m, dtype=torch.float64).reshape(-1).to("cuda")

    def solve(self, Fs, Bs):
        return self.helm.solve_batch(Fs, Bs, tol=self.tol, stream=self.solve_stream)

    def release(self, F):
        F.close()

    def sync(self):
        import torch
        if self.own is not None:
            self.own.synchronize()
        else:
            torch.cuda.synchronize()


def _grid_key(grid, precision=None):
    return tuple(getattr(grid, a, None) for a in ("nx", "nz", "hx", "hz")) + (precision,)


class Server:
    """Continuous batching.  A batch holds requests on one grid: the oldest
    queued request leads it and later requests on the same grid join it in
    arrival order, passing requests on other grids (a batch's launch chain
    is as long as its largest system, so a mixed batch makes every request
    wait for the largest).  A request passed max_overtakes times is not
    passed again (max_overtakes = 0: first in, first out, one grid per
    batch; None: first in, first out with grids mixed in a batch)."""

    def __init__(self, backend, hbm_budget: int, max_chains: int = MAX_CHAINS, resident: bool = False,
                 clock=time.perf_counter, max_overtakes=4):
        if max_chains < 1 or max_chains > MAX_CHAINS:
            raise ValueError(f"max_chains must be in [1, {MAX_CHAINS}]")
        if max_overtakes is not None and max_overtakes < 0:
            raise ValueError("max_overtakes must be >= 0 or None")
        self.max_overtakes = None if max_overtakes is None else int(max_overtakes)
        self.overtaken = {}              # rid -> times passed by a later request
        self.be = backend
        self.budget = int(hbm_budget)
        self.max_chains = max_chains
        self.resident = resident
        self.clock = clock
        self.queue = collections.deque()
        self.cache = collections.OrderedDict()     # (key, omega) -> (factor, bytes)
        self.cache_bytes = 0
        self.batches = 0
        self.rejected = []
        self.inflight_bytes = 0          # batches admitted and not finished (pipelined and lane runs)
        self.inflight_keys = set()
        self._inflight = []              # lane runs: the batches in flight

    # -- memory accounting --------------------------------------------------
    def _prec(self, req: ServeRequest):
        """The request's precision (its own, else the backend's)."""
        return req.precision if req.precision is not None else getattr(self.be, "precision", None)

    def _fkey(self, req: ServeRequest, w):
        """Key of a resident factor: model, frequency and precision."""
        return (req.model_key, float(w), self._prec(req))

    def _fbytes(self, req: ServeRequest) -> int:
        p = self._prec(req)
        return self.be.factor_bytes(req.grid, p) if req.precision is not None else self.be.factor_bytes(req.grid)

    def _need(self, req: ServeRequest, reuse) -> int:
        fb = self._fbytes(req)
        n_new = sum(1 for w in req.omegas if self._fkey(req, w) not in reuse)
        return n_new * fb + len(req.omegas) * BYTES_PER_UNKNOWN_RHS * req.grid.N * req.S

    def _evict(self, need: int, keep) -> bool:
        """Free resident factors (least recently used first, never those in
        `keep`) until `need` more bytes fit.  Returns whether they fit."""
        while self.cache_bytes + need > self.budget:
            victim = next((k for k in self.cache if k not in keep), None)
            if victim is None:
                return False
            F, b = self.cache.pop(victim)
            self.be.release(F)
            self.cache_bytes -= b
        return True

    # -- queue --------------------------------------------------------------
    def submit(self, req: ServeRequest):
        if len(req.omegas) > self.max_chains:
            raise ValueError(f"request {req.rid}: {len(req.omegas)} frequencies exceed {self.max_chains} chains")
        alone = self._need(req, ())
        if alone > self.budget:
            self.rejected.append(req.rid)
            raise MemoryError(f"request {req.rid} needs {alone} bytes, above the HBM budget {self.budget}")
        self.queue.append(req)

    def admit(self):
        """Requests of the next batch: the oldest request and the later ones
        on its grid, in arrival order, within the chain and memory limits
        (memory of a batch still in flight counts against the budget, and
        the resident factors it uses are not evicted).  The scan stops at the
        first request that does not fit, and at a request on another grid
        that has been passed max_overtakes times."""
        batch, chains, used = [], 0, self.inflight_bytes
        keep = set(self.inflight_keys)
        if not self.queue:
            return batch
        gk = _grid_key(self.queue[0].grid, self._prec(self.queue[0]))
        taken = []
        for idx, req in enumerate(self.queue):
            if self.max_overtakes is None:
                if self._prec(req) != gk[-1]:
                    break              # first in, first out: a batch has one precision
            elif _grid_key(req.grid, self._prec(req)) != gk:
                if self.overtaken.get(req.rid, 0) >= self.max_overtakes:
                    break
                continue
            if chains + len(req.omegas) > self.max_chains:
                break
            keys = {self._fkey(req, w) for w in req.omegas} if req.model_key is not None else set()
            hit = {k for k in keys if k in self.cache}
            need = self._need(req, hit)
            if not self._evict(used + need, keep | hit):
                break
            keep |= hit
            batch.append(req)
            taken.append(idx)
            chains += len(req.omegas)
            used += need
        if taken:
            tset = set(taken)
            for idx in range(taken[-1]):
                if idx not in tset:
                    rid = self.queue[idx].rid
                    self.overtaken[rid] = self.overtaken.get(rid, 0) + 1
            self.queue = collections.deque(r for i, r in enumerate(self.queue) if i not in tset)
            for r in batch:
                self.overtaken.pop(r.rid, None)
        return batch

    def _track(self, prep: "_Prepared", add: bool):
        """Count a lane's batch in flight (or no longer): its memory and the
        resident factors it uses are protected until it finishes."""
        if add:
            self._inflight.append(prep)
        else:
            self._inflight.remove(prep)
        self.inflight_bytes = sum(p.bytes for p in self._inflight)
        self.inflight_keys = set().union(*[p.keys for p in self._inflight])

    def _begin(self, batch, be=None, rhs=True) -> "_Prepared":
        """Bookkeeping of an admitted batch: resident factors it reuses, the
        systems to factor, and (rhs=True) its right-hand sides (host thread of
        the caller; `be`: the lane that runs it, by default the server's
        backend).  rhs=False leaves the right-hand sides to _rhs, which needs
        no lock."""
        prep = _Prepared(batch, self.clock())
        prep.be = be if be is not None else self.be
        prep.precision = batch[0].precision
        for r, req in enumerate(batch):
            m = prep.be.model(req)
            for q, w in enumerate(req.omegas):
                key = self._fkey(req, w)
                if req.model_key is not None and key in self.cache:
                    self.cache.move_to_end(key)
                    prep.Fs[(r, q)] = self.cache[key][0]
                    prep.keys.add(key)
                else:
                    prep.grids.append(req.grid)
                    prep.ms.append(m)
                    prep.oms.append(float(w))
                    prep.slots.append((r, q))
            prep.bytes += self._need(req, prep.keys)
        if rhs:
            self._rhs(prep)
        return prep

    def _rhs(self, prep: "_Prepared"):
        """The batch's right-hand sides, on its lane, complete on return."""
        prep.Bs = {r: prep.be.rhs(req) for r, req in enumerate(prep.batch)}
        prep.be.sync()

    def _factor(self, prep: "_Prepared"):
        if prep.grids:
            Fs = (prep.be.factor(prep.grids, prep.ms, prep.oms, prep.precision) if prep.precision is not None
                  else prep.be.factor(prep.grids, prep.ms, prep.oms))
            for slot, F in zip(prep.slots, Fs):
                prep.Fs[slot] = F

    def _solve(self, prep: "_Prepared"):
        order = [(r, q) for r, req in enumerate(prep.batch) for q in range(len(req.omegas))]
        X, infos = prep.be.solve([prep.Fs[k] for k in order], [prep.Bs[k[0]] for k in order])
        prep.be.sync()
        return X, infos

    def _finish(self, prep: "_Prepared", X, infos):
        t1 = self.clock()
        out, c = [], 0
        for r, req in enumerate(prep.batch):
            k = len(req.omegas)
            out.append(ServeResult(req.rid, X[c:c + k], infos[c:c + k], req.arrival, prep.t0, t1, self.batches))
            c += k
        # keep or free the factors made for this batch
        for r, q in prep.slots:
            req = prep.batch[r]
            F = prep.Fs[(r, q)]
            key = self._fkey(req, req.omegas[q])
            if self.resident and req.model_key is not None and key not in self.cache:
                b = self._fbytes(req)
                if self._evict(b, set(self.inflight_keys)):
                    self.cache[key] = (F, b)
                    self.cache_bytes += b
                    continue
            self.be.release(F)
        self.batches += 1
        return out

    def step(self):
        """Run one batch; returns its results (empty if the queue is empty)."""
        batch = self.admit()
        if not batch:
            return []
        prep = self._begin(batch)
        self._factor(prep)
        X, infos = self._solve(prep)
        return self._finish(prep, X, infos)

    def close(self):
        for F, _ in self.cache.values():
            self.be.release(F)
        self.cache.clear()
        self.cache_bytes = 0


def run_stream(server: Server, requests, realtime: bool = True, pipelined: bool = False):
    """Feed `requests` (sorted by arrival) to the server as they arrive and
    run it until all are done.  Returns the results in completion order.

    pipelined: while one batch is solved, the next admitted batch is
    factored (on the backend's factor stream, from a second host thread);
    the admission counts the memory of the batch in flight."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    results = []
    t0 = server.clock()

    def arrivals():
        now = server.clock() - t0 if realtime else math.inf
        while pending and pending[0].arrival <= now:
            server.submit(pending.popleft())

    def collect(out):
        for res in out:
            res.start -= t0
            res.done -= t0
            results.append(res)

    if not pipelined:
        while pending or server.queue:
            arrivals()
            if not server.queue:
                if pending and realtime:
                    time.sleep(max(0.0, pending[0].arrival - (server.clock() - t0)))
                continue
            collect(server.step())
        return results

    inflight = None
    while pending or server.queue or inflight is not None:
        arrivals()
        batch = server.admit() if server.queue else []
        nxt = server._begin(batch) if batch else None
        if inflight is None and nxt is None:
            if pending and realtime:
                time.sleep(max(0.0, pending[0].arrival - (server.clock() - t0)))
            continue
        err = []

        def factor_next():
            try:
                server._factor(nxt)
            except BaseException as e:      # re-raised below
                err.append(e)

        th = None
        if nxt is not None:
            th = threading.Thread(target=factor_next)
            th.start()
        solved = server._solve(inflight) if inflight is not None else None
        if th is not None:
            th.join()
        if err:
            raise err[0]
        # from here the batch in flight is nxt: its memory and resident
        # factors are protected while the finished batch's factors are
        # cached or released
        server.inflight_bytes = nxt.bytes if nxt is not None else 0
        server.inflight_keys = set(nxt.keys) if nxt is not None else set()
        if inflight is not None:
            collect(server._finish(inflight, *solved))
        inflight = nxt
    return results


def run_lanes(server: Server, requests, lanes: int = 2, realtime: bool = True):
    """Feed `requests` (sorted by arrival) to the server and run `lanes`
    batches side by side until all are done; results in completion order.

    Each lane is a host thread with a backend of its own (backend.lane(k):
    one stream).  A free lane admits the next batch (the server's admission
    rules, with the memory of every batch in flight counted against the
    budget), factors and solves it, and hands the results back.  Admission,
    the resident-factor cache and the results are shared under one lock; the
    factorisations and solves run outside it (the library calls release the
    interpreter lock).  A lane with nothing to admit waits until a batch
    finishes or the next request arrives; it stops when no request is
    pending or queued."""
    if lanes < 1:
        raise ValueError("lanes must be >= 1")
    if not callable(getattr(server.be, "lane", None)):
        raise TypeError("run_lanes needs a backend with lane(k) (a backend per lane, on a stream of its own)")
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    results, err = [], []
    cv = threading.Condition()
    t0 = server.clock()
    backends = [server.be.lane(k) for k in range(lanes)]

    def arrivals():
        now = server.clock() - t0 if realtime else math.inf
        while pending and pending[0].arrival <= now:
            server.submit(pending.popleft())

    def lane(be):
        ctx = be.stream_context() if hasattr(be, "stream_context") else None
        if ctx is not None:
            ctx.__enter__()
        try:
            while True:
                with cv:
                    while True:
                        if err:
                            return
                        arrivals()
                        batch = server.admit() if server.queue else []
                        if batch:
                            prep = server._begin(batch, be, rhs=False)
                            server._track(prep, True)
                            break
                        if not pending and not server.queue:
                            return
                        wait = None
                        if pending and realtime:
                            wait = max(0.0, pending[0].arrival - (server.clock() - t0))
                        cv.wait(wait)
                try:
                    server._rhs(prep)                # outside the lock
                    server._factor(prep)
                    X, infos = server._solve(prep)
                except BaseException as e:      # re-raised on the calling thread
                    with cv:
                        err.append(e)
                        server._track(prep, False)
                        for F in prep.Fs.values():
                            if not any(F is c[0] for c in server.cache.values()):
                                server.be.release(F)
                        cv.notify_all()
                    return
                with cv:
                    server._track(prep, False)
                    for res in server._finish(prep, X, infos):
                        res.start -= t0
                        res.done -= t0
                        results.append(res)
                    cv.notify_all()
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)

    threads = [threading.Thread(target=lane, args=(be,)) for be in backends]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if err:
        raise err[0]
    return results


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def summary(results, requests) -> dict:
    """Latency percentiles and rates of a finished stream.  The offered and
    served rates count the same n - 1 intervals: between the first and last
    arrival, and between the first and last completion, so the drain of the
    last requests does not count against a server that keeps up.  The queue
    is stable when the service keeps pace (served >= 0.95 offered);
    latency_growth (median latency of the last quarter of arrivals over that
    of the first quarter) shows a queue that builds up."""
    lat = [r.latency for r in results]
    n = len(results)
    span = max(r.done for r in results) - min(q.arrival for q in requests)
    solves = sum(q.S * len(q.omegas) for q in requests)
    arr = sorted(q.arrival for q in requests)
    done = sorted(r.done for r in results)
    offered = (len(arr) - 1) / max(1e-12, arr[-1] - arr[0]) if len(arr) > 1 else 0.0
    served = (n - 1) / max(1e-12, done[-1] - done[0]) if n > 1 else 0.0
    by_arrival = [r.latency for r in sorted(results, key=lambda r: r.arrival)]
    q = max(1, n // 4)
    growth = percentile(by_arrival[-q:], 0.5) / max(1e-12, percentile(by_arrival[:q], 0.5))
    return {"requests": n, "p50_ms": percentile(lat, 0.5) * 1e3, "p99_ms": percentile(lat, 0.99) * 1e3,
            "max_ms": max(lat) * 1e3, "solves_per_s": solves / span, "offered_req_per_s": offered,
            "served_req_per_s": served, "stable": served >= 0.95 * offered, "latency_growth": growth,
            "batches": len({r.batch for r in results})}


def run_c5(requests: int = 32, rate: float = 200.0, seed: int = 0, budget_gb: float = 64.0,
           precision: str = "fp32_ir", max_chains: int = MAX_CHAINS, serial: bool = False, max_overtakes=4,
           lanes: int = 0) -> dict:
    """The serving workload (Poisson arrivals of single-frequency requests,
    n in {101, 201, 301, 401}, 8 to 128 sources, each with its own seeded
    layered model) through the server; returns the summary.  lanes > 0:
    run_lanes with that many lanes (else the pipelined or serial loop)."""
    import torch
    from . import helm
    from . import inputs as I

    stream = I.serving_stream(requests, rate, seed)
    reqs = []
    for q in stream:
        m, omega, src = I.request_inputs(q)
        g = helm.Grid(q.n, q.n, I.H_KM, I.H_KM)
        reqs.append(ServeRequest(q.rid, g, torch.as_tensor(m.reshape(-1), device="cuda"), [omega], list(src),
                                 arrival=q.t_arrival))
    be = HelmBackend(precision, 1e-10, stream=pooled_stream("factor"), solve_stream=pooled_stream("solve"))
    srv = Server(be, int(budget_gb * 2**30), max_chains, max_overtakes=max_overtakes)
    # warm-up: one small request through the whole path
    warm = ServeRequest(-1, helm.Grid(33, 33, I.H_KM, I.H_KM), torch.full((33 * 33,), 0.25, device="cuda",
                        dtype=torch.float64), [1.0], [5])
    srv.submit(warm)
    srv.step()
    torch.cuda.synchronize()
    if lanes > 0:
        res = run_lanes(srv, reqs, lanes)
        sched = f"{lanes} lanes"
    else:
        res = run_stream(srv, reqs, pipelined=not serial)
        sched = "serial" if serial else "pipelined"
    worst = max(i.max_relres for r in res for i in r.infos)
    out = summary(res, reqs)
    out.update({"precision": precision, "max_relres": worst, "budget_gb": budget_gb,
                "schedule": sched,
                "admission": "mixed grids, first in first out" if max_overtakes is None else
                             f"one grid per batch, a request passed at most {max_overtakes} times",
                "rate": rate, "sizes": sorted({q.n for q in stream})})
    srv.close()
    return out


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--requests", type=int, default=32)
    p.add_argument("--rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--budget-gb", type=float, default=64.0)
    p.add_argument("--precision", default="fp32_ir", choices=["fp32_ir", "fp64"])
    p.add_argument("--max-chains", type=int, default=MAX_CHAINS)
    p.add_argument("--max-overtakes", type=int, default=4,
                   help="times a request may be passed by later requests on the batch's grid (-1: grids mixed, "
                        "first in, first out)")
    p.add_argument("--serial", action="store_true",
                   help="one batch at a time (default: the next batch is factored while the current is solved)")
    p.add_argument("--lanes", type=int, default=0,
                   help="batches run side by side, each factored and solved on a stream of its own (0: the "
                        "pipelined or serial loop)")
    args = p.parse_args(argv)
    out = run_c5(args.requests, args.rate, args.seed, args.budget_gb, args.precision, args.max_chains, args.serial,
                 None if args.max_overtakes < 0 else args.max_overtakes, args.lanes)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
