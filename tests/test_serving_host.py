"""Scheduler logic of the serving layer, on the CPU with a stand-in backend
(no device work): FIFO admission, the chain and HBM limits, rejection,
resident factors and their eviction, and that no factor leaks."""
import dataclasses

import pytest

from paper_2301_10762_amd import serving as SV


@dataclasses.dataclass(frozen=True)
class G:
    nx: int
    nz: int

    @property
    def N(self):
        return self.nx * self.nz


class FakeFactor:
    def __init__(self, ident, grid, omega):
        self.ident, self.grid, self.omega, self.live = ident, grid, omega, True


class FakeInfo:
    max_relres = 0.0


class FakeBackend:
    """factor bytes = 100 per unknown; solutions = the factor identities."""

    def __init__(self):
        self.made, self.calls = [], []

    def factor_bytes(self, grid, precision=None):
        return (50 if precision == "fp32_ir" else 100) * grid.N

    def factor(self, grids, ms, omegas, precision=None):
        self.calls.append(len(grids))
        self.precisions = getattr(self, "precisions", []) + [precision]
        out = [FakeFactor(len(self.made) + c, g, w) for c, (g, w) in enumerate(zip(grids, omegas))]
        self.made += out
        self.max_live = max(getattr(self, "max_live", 0), self.live())
        return out

    def rhs(self, req):
        return ("B", req.rid)

    def model(self, req):
        return req.m

    def solve(self, Fs, Bs):
        assert all(F.live for F in Fs)
        return [(F.ident, B) for F, B in zip(Fs, Bs)], [FakeInfo() for _ in Fs]

    def release(self, F):
        assert F.live
        F.live = False

    def sync(self):
        pass

    def live(self):
        return sum(F.live for F in self.made)


def req(rid, n=10, omegas=(1.0,), S=4, key=None, arrival=0.0):
    return SV.ServeRequest(rid, G(n, n), None, list(omegas), list(range(S)), arrival=arrival, model_key=key)


def per_request_bytes(n, S, n_omega=1):
    return n_omega * (100 * n * n + SV.BYTES_PER_UNKNOWN_RHS * n * n * S)


def test_fifo_batches_respect_chain_limit():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16)
    for r in range(20):
        srv.submit(req(r))
    first = srv.step()
    second = srv.step()
    assert [x.rid for x in first] == list(range(16))
    assert [x.rid for x in second] == list(range(16, 20))
    assert be.calls == [16, 4] and be.live() == 0
    assert srv.step() == []


def test_multi_frequency_requests_count_one_chain_per_frequency():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16)
    srv.submit(req(0, omegas=(1.0, 2.0, 3.0, 4.0, 5.0)))
    srv.submit(req(1, omegas=(1.0,) * 10))
    srv.submit(req(2, omegas=(1.0, 2.0)))
    b1 = srv.step()
    assert [x.rid for x in b1] == [0, 1]            # 15 chains; request 2 would make 17
    assert len(b1[0].X) == 5 and len(b1[1].X) == 10
    assert [x.rid for x in srv.step()] == [2]
    with pytest.raises(ValueError):
        srv.submit(req(3, omegas=(1.0,) * 17))


def test_memory_budget_limits_batches_and_rejects_oversize():
    be = FakeBackend()
    one = per_request_bytes(10, 4)
    srv = SV.Server(be, 2 * one + one // 2, max_chains=16)
    for r in range(5):
        srv.submit(req(r))
    sizes = []
    while True:
        b = srv.step()
        if not b:
            break
        sizes.append(len(b))
    assert sizes == [2, 2, 1] and be.live() == 0
    with pytest.raises(MemoryError):
        srv.submit(req(9, n=40))
    assert srv.rejected == [9]


def test_head_of_line_request_is_not_overtaken():
    """Strict first in, first out (max_overtakes = 0)."""
    be = FakeBackend()
    small, big = per_request_bytes(10, 4), per_request_bytes(20, 4)
    srv = SV.Server(be, big + small // 2, max_chains=16, max_overtakes=0)
    srv.submit(req(0, n=10))
    srv.submit(req(1, n=20))
    srv.submit(req(2, n=10))
    assert [x.rid for x in srv.step()] == [0]       # 1 does not fit beside 0; 2 must wait behind 1
    assert [x.rid for x in srv.step()] == [1]
    assert [x.rid for x in srv.step()] == [2]


def test_batches_hold_one_grid_and_pass_other_grids():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16)
    for rid, n in enumerate((10, 20, 10, 20, 10)):
        srv.submit(req(rid, n=n))
    assert [x.rid for x in srv.step()] == [0, 2, 4]
    assert [x.rid for x in srv.step()] == [1, 3]
    assert srv.step() == [] and be.live() == 0


def test_passing_is_bounded():
    """A request already passed max_overtakes times stops the scan; the
    count grows each time a later request joins a batch ahead of it."""
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16, max_overtakes=2)
    for rid, n in enumerate((10, 20, 10)):
        srv.submit(req(rid, n=n))
    srv.overtaken[1] = 2
    assert [x.rid for x in srv.step()] == [0]
    assert [x.rid for x in srv.step()] == [1]
    assert [x.rid for x in srv.step()] == [2]
    srv2 = SV.Server(FakeBackend(), 1 << 40, max_chains=16, max_overtakes=2)
    for rid, n in enumerate((10, 20, 10)):
        srv2.submit(req(rid, n=n))
    assert [x.rid for x in srv2.step()] == [0, 2]
    assert srv2.overtaken == {1: 1}
    assert [x.rid for x in srv2.step()] == [1] and srv2.overtaken == {}


def test_mixed_grid_fifo_mode():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16, max_overtakes=None)
    for rid, n in enumerate((10, 20, 10)):
        srv.submit(req(rid, n=n))
    assert [x.rid for x in srv.step()] == [0, 1, 2]


def test_resident_factors_are_reused_and_evicted_lru():
    be = FakeBackend()
    fb = 100 * 100
    work = SV.BYTES_PER_UNKNOWN_RHS * 100 * 4
    srv = SV.Server(be, 2 * fb + work, max_chains=16, resident=True)
    srv.submit(req(0, key="a"))
    r0 = srv.step()[0]
    srv.submit(req(1, key="a"))
    r1 = srv.step()[0]
    assert be.calls == [1]                          # second request reused the factor
    assert r1.X[0][0] == r0.X[0][0]
    assert srv.cache_bytes == fb and be.live() == 1
    srv.submit(req(2, key="b"))
    srv.step()
    assert set(k[0] for k in srv.cache) == {"a", "b"}
    srv.submit(req(3, key="c"))                     # needs room: "a" is least recently used
    srv.step()
    assert set(k[0] for k in srv.cache) == {"b", "c"}
    assert be.live() == 2
    srv.close()
    assert be.live() == 0 and srv.cache_bytes == 0


def test_same_key_twice_in_one_batch_does_not_leak():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=16, resident=True)
    srv.submit(req(0, key="a"))
    srv.submit(req(1, key="a"))
    srv.step()
    assert len(srv.cache) == 1 and be.live() == 1
    srv.close()
    assert be.live() == 0


def test_run_stream_serves_everything_and_summarises():
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=4)
    reqs = [req(r, arrival=0.001 * r) for r in range(10)]
    res = SV.run_stream(srv, reqs, realtime=False)
    assert sorted(x.rid for x in res) == list(range(10))
    s = SV.summary(res, reqs)
    assert s["requests"] == 10 and s["batches"] == 3
    assert s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]


def test_pipelined_stream_serves_everything_without_leaks():
    """Two batches in flight: every request is served once, resident
    factors are reused, and no factor is leaked or released twice."""
    be = FakeBackend()
    srv = SV.Server(be, 1 << 40, max_chains=4, resident=True)
    reqs = [req(r, key=("k", r % 3), arrival=0.001 * r) for r in range(12)]
    res = SV.run_stream(srv, reqs, realtime=False, pipelined=True)
    assert sorted(x.rid for x in res) == list(range(12))
    assert srv.inflight_bytes == 0 and not srv.inflight_keys
    assert be.live() == len(srv.cache) == 3
    srv.close()
    assert be.live() == 0


def test_pipelined_admission_counts_the_batch_in_flight():
    """With room for two requests in all, a batch of two cannot be followed
    by another while it is in flight: batches alternate with the solves."""
    be = FakeBackend()
    one = per_request_bytes(10, 4)
    srv = SV.Server(be, 2 * one + one // 2, max_chains=16)
    reqs = [req(r, arrival=0.0) for r in range(5)]
    res = SV.run_stream(srv, reqs, realtime=False, pipelined=True)
    assert sorted(x.rid for x in res) == list(range(5))
    sizes = [len([x for x in res if x.batch == b]) for b in sorted({x.batch for x in res})]
    assert sum(sizes) == 5 and max(sizes) <= 2
    assert be.max_live <= 2                         # never a second batch beside the one in flight
    assert be.live() == 0


class LaneFake(FakeBackend):
    """Stand-in whose solves take a little time and record how many run at
    once; every lane shares it."""

    def __init__(self, delay=0.03):
        super().__init__()
        import threading
        self.delay, self.busy, self.max_busy = delay, 0, 0
        self.lock = threading.Lock()

    def lane(self, k=0):
        return self

    def solve(self, Fs, Bs):
        import time
        with self.lock:
            self.busy += 1
            self.max_busy = max(self.max_busy, self.busy)
        time.sleep(self.delay)
        with self.lock:
            self.busy -= 1
        return super().solve(Fs, Bs)


def test_lanes_run_batches_side_by_side():
    """Two grids queued at once and two lanes: the two batches (one grid
    each) are solved at the same time."""
    be = LaneFake()
    srv = SV.Server(be, 1 << 40, max_chains=16)
    reqs = [req(r, n=10 + 5 * (r % 2), arrival=0.0) for r in range(8)]
    res = SV.run_lanes(srv, reqs, lanes=2, realtime=False)
    assert sorted(x.rid for x in res) == list(range(8))
    assert be.max_busy == 2
    for b in {x.batch for x in res}:
        assert len({x.rid % 2 for x in res if x.batch == b}) == 1     # one grid per batch
    assert srv.inflight_bytes == 0 and not srv.inflight_keys
    assert be.live() == 0


def test_lanes_serve_everything_without_leaks():
    """Three lanes with resident factors: every request is served once,
    factors are reused, and none is leaked or released twice."""
    be = LaneFake(delay=0.005)
    srv = SV.Server(be, 1 << 40, max_chains=4, resident=True)
    reqs = [req(r, key=("k", r % 3), arrival=0.001 * r) for r in range(15)]
    res = SV.run_lanes(srv, reqs, lanes=3, realtime=False)
    assert sorted(x.rid for x in res) == list(range(15))
    assert all(x.X[0][1] == ("B", x.rid) for x in res)
    assert srv.inflight_bytes == 0 and not srv.inflight_keys
    assert be.live() == len(srv.cache) == 3
    srv.close()
    assert be.live() == 0


def test_lanes_admission_counts_every_batch_in_flight():
    """With room for two requests in all, three lanes never hold more than
    two requests' factors at once."""
    be = LaneFake(delay=0.01)
    one = per_request_bytes(10, 4)
    srv = SV.Server(be, 2 * one + one // 2, max_chains=16)
    reqs = [req(r, arrival=0.0) for r in range(7)]
    res = SV.run_lanes(srv, reqs, lanes=3, realtime=False)
    assert sorted(x.rid for x in res) == list(range(7))
    assert be.max_live <= 2
    assert be.live() == 0


def test_lanes_realtime_waits_for_arrivals():
    """Requests arriving over time are all served; none starts before it
    arrives."""
    be = LaneFake(delay=0.002)
    srv = SV.Server(be, 1 << 40, max_chains=4)
    reqs = [req(r, n=10 + 5 * (r % 3), arrival=0.004 * r) for r in range(10)]
    res = SV.run_lanes(srv, reqs, lanes=2, realtime=True)
    assert sorted(x.rid for x in res) == list(range(10))
    assert all(x.start >= x.arrival - 1e-9 for x in res)
    assert be.live() == 0


def test_lanes_reraise_backend_errors_without_leaks():
    class Failing(LaneFake):
        def solve(self, Fs, Bs):
            raise RuntimeError("device error")

    be = Failing()
    srv = SV.Server(be, 1 << 40, max_chains=2)
    with pytest.raises(RuntimeError, match="device error"):
        SV.run_lanes(srv, [req(r) for r in range(4)], lanes=2, realtime=False)
    assert be.live() == 0
    assert srv.inflight_bytes == 0


def _res(rid, arrival, done):
    return SV.ServeResult(rid, [], [], arrival, arrival, done, rid)


def test_summary_rates_keep_pace_and_growing_queue():
    """A server that finishes every request a fixed 50 ms after it arrives
    keeps pace (served = offered, no latency growth); one that finishes a
    request every 20 ms against arrivals every 10 ms does not."""
    reqs = [req(r, arrival=0.01 * r) for r in range(40)]
    s = SV.summary([_res(r, 0.01 * r, 0.01 * r + 0.05) for r in range(40)], reqs)
    assert s["offered_req_per_s"] == pytest.approx(100.0)
    assert s["served_req_per_s"] == pytest.approx(100.0)
    assert s["stable"] and s["latency_growth"] == pytest.approx(1.0)
    s = SV.summary([_res(r, 0.01 * r, 0.05 + 0.02 * r) for r in range(40)], reqs)
    assert s["served_req_per_s"] == pytest.approx(50.0)
    assert not s["stable"] and s["latency_growth"] > 3.0


def test_lanes_need_a_backend_with_lanes():
    srv = SV.Server(FakeBackend(), 1 << 40)
    with pytest.raises(TypeError, match="lane"):
        SV.run_lanes(srv, [req(0)], lanes=2, realtime=False)
    with pytest.raises(ValueError):
        SV.run_lanes(SV.Server(LaneFake(), 1 << 40), [req(0)], lanes=0, realtime=False)


def test_batches_have_one_precision():
    """Requests naming different precisions never share a batch (first in,
    first out or grouped by grid); each batch is factored in its requests'
    precision and counted with that precision's factor size."""
    for overtakes in (None, 4):
        be = FakeBackend()
        srv = SV.Server(be, 1 << 40, max_chains=16, max_overtakes=overtakes)
        precs = ["fp64", "fp64", "fp32_ir", "fp64", "fp32_ir", "fp32_ir"]
        for r, p in enumerate(precs):
            q = req(r)
            q.precision = p
            srv.submit(q)
        batches = []
        while srv.queue:
            out = srv.step()
            batches.append(sorted(x.rid for x in out))
        for b, p in zip(batches, be.precisions):
            assert {precs[r] for r in b} == {p}, (overtakes, batches, be.precisions)
        assert sorted(r for b in batches for r in b) == list(range(len(precs)))
        if overtakes is None:
            assert batches == [[0, 1], [2], [3], [4, 5]]
        else:
            assert batches == [[0, 1, 3], [2, 4, 5]]
    srv = SV.Server(FakeBackend(), 1 << 40)
    q = req(9, n=10, S=4)
    q.precision = "fp32_ir"
    assert srv._need(q, set()) == 50 * 100 + SV.BYTES_PER_UNKNOWN_RHS * 100 * 4
