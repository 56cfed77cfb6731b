"""GPU: the serving layer and the autograd wrapper, through the C ABI.

Serving: a request's solutions are bitwise the same whether it is served
alone or batched with other requests (chains are independent in every
launch), and match the FP64 oracle; resident factors are reused.
Autograd: phi and its backward equal the oracle's misfit and gradient, and
torch.autograd.gradcheck passes on a 9 x 9 grid.
"""
import numpy as np
import pytest

import oracle
from tests.parity import assert_cols, rel
from paper_2301_10762_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    return h


# (n, model seed, points per wavelength of each frequency, sources)
SPECS = [(17, 1, (9.0, 12.0), 3), (33, 2, (10.0,), 5), (40, 3, (8.0, 11.0, 14.0), 8), (21, 4, (12.0,), 2)]


def make_request(SV, helm, rid, n, seed, ppws, n_src, key=None):
    m = I.layered_model(n, seed)
    omegas = [I.omega_from_ppw(p, I.C_MIN, I.H_KM) for p in ppws]
    src = [int(k) for k in I.surface_sources(n, n_src, depth=2, margin=(1, n - 2))]
    g = helm.Grid(n, n, I.H_KM, I.H_KM)
    return SV.ServeRequest(rid, g, torch.as_tensor(m.reshape(-1), device="cuda"), omegas, src, model_key=key), m


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_serving_alone_equals_mixed_and_matches_oracle(helm, precision):
    from paper_2301_10762_amd import serving as SV
    alone = {}
    for rid, spec in enumerate(SPECS):
        print(f"alone: request {rid} {spec}", flush=True)
        be = SV.HelmBackend(precision, 1e-10)
        srv = SV.Server(be, 1 << 36)
        req, _ = make_request(SV, helm, rid, *spec)
        srv.submit(req)
        res = srv.step()
        assert len(res) == 1
        alone[rid] = [x.clone() for x in res[0].X]
    be = SV.HelmBackend(precision, 1e-10)
    srv = SV.Server(be, 1 << 36, max_overtakes=None)       # every grid in one batch
    models = {}
    for rid, spec in enumerate(SPECS):
        req, models[rid] = make_request(SV, helm, rid, *spec)
        srv.submit(req)
    print("mixed batch", flush=True)
    res = srv.step()
    assert sorted(r.rid for r in res) == list(range(len(SPECS))) and srv.batches == 1
    for r in res:
        n, _, ppws, n_src = SPECS[r.rid]
        assert max(i.max_relres for i in r.infos) <= 1e-10
        for q, X in enumerate(r.X):
            assert torch.equal(X, alone[r.rid][q]), (r.rid, q)
        g = oracle.Grid(n, n, I.H_KM, I.H_KM)
        src = I.surface_sources(n, n_src, depth=2, margin=(1, n - 2))
        for q, p in enumerate(ppws):
            w = I.omega_from_ppw(p, I.C_MIN, I.H_KM)
            F = oracle.Factor(g, models[r.rid], w)
            Xo = F.solve(oracle.unit_sources(g, src))
            F.close()
            assert_cols(r.X[q].cpu().numpy(), Xo, 1e-9, what=f"request {r.rid}, frequency {q}")


@pytest.mark.parametrize("lanes", [0, 3])
def test_mixed_precision_stream_equals_alone(helm, lanes):
    """Requests that name their own precision (complex128, or complex64 +
    FP64 refinement) in one stream: batches are formed per grid and
    precision, and every result is bitwise the one of the same request
    served alone in its precision, with the serial loop and with lanes."""
    from paper_2301_10762_amd import serving as SV
    precs = ["fp64", "fp32_ir", "fp32_ir", "fp64"]
    alone = {}
    for rid, (spec, p) in enumerate(zip(SPECS, precs)):
        srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36)
        req, _ = make_request(SV, helm, rid, *spec)
        req.precision = p
        srv.submit(req)
        alone[rid] = [x.clone() for x in srv.step()[0].X]
    reqs = []
    for rid, (spec, p) in enumerate(zip(SPECS + SPECS, precs + precs[::-1])):
        req, _ = make_request(SV, helm, rid % len(SPECS) + 10 * (rid // len(SPECS)), *spec)
        req.precision = p
        reqs.append(req)
    # the second copy of each spec asks for the other precision: its solo result
    for rid, (spec, p) in enumerate(zip(SPECS, precs[::-1])):
        srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36)
        req, _ = make_request(SV, helm, 10 + rid, *spec)
        req.precision = p
        srv.submit(req)
        alone[10 + rid] = [x.clone() for x in srv.step()[0].X]
    srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36, max_chains=8)
    print(f"mixed-precision stream, lanes {lanes}", flush=True)
    res = SV.run_lanes(srv, reqs, lanes=lanes, realtime=False) if lanes else SV.run_stream(srv, reqs, realtime=False)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == sorted(alone)
    for r in res:
        assert max(i.max_relres for i in r.infos) <= 1e-10
        for q, X in enumerate(r.X):
            assert torch.equal(X, alone[r.rid][q]), (r.rid, q)
    srv.close()


def test_serving_resident_factors_reused(helm):
    from paper_2301_10762_amd import serving as SV
    be = SV.HelmBackend("fp64", 1e-10)
    srv = SV.Server(be, 1 << 36, resident=True)
    r0, _ = make_request(SV, helm, 0, 33, 7, (10.0, 12.0), 4, key="m7")
    srv.submit(r0)
    a = srv.step()[0]
    made = be.factorisations
    r1, _ = make_request(SV, helm, 1, 33, 7, (10.0, 12.0), 4, key="m7")
    srv.submit(r1)
    b = srv.step()[0]
    assert be.factorisations == made == 2
    for x, y in zip(a.X, b.X):
        assert torch.equal(x, y)
    srv.close()
    assert srv.cache_bytes == 0


def _tiny_fwi(n=9, seed=5):
    w = I.small_layered(n, seed, 2, 3, ppws=(6.0,))
    g = oracle.Grid.of(w)
    d_obs = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    return w, g, d_obs


def test_autograd_matches_oracle(helm):
    from paper_2301_10762_amd.autograd import misfit
    w, g, d_obs = _tiny_fwi(15, 6)
    phi_o, grad_o = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers, 1e-4, 1e-6)
    m = torch.as_tensor(w.m.reshape(w.nz, w.nx), device="cuda").clone().requires_grad_(True)
    loss = 3.0 * misfit(m, helm.Grid.of(w), w.omegas, d_obs, w.sources, w.receivers, 1e-4, 1e-6, "fp64", 1e-10)
    loss.backward()
    assert abs(loss.item() / 3.0 - phi_o) / phi_o < 1e-10
    assert m.grad.shape == (w.nz, w.nx)
    assert rel(m.grad.cpu().numpy().reshape(-1) / 3.0, grad_o) < 1e-8


def test_autograd_gradcheck(helm):
    from paper_2301_10762_amd.autograd import misfit
    w, g, d_obs = _tiny_fwi()
    G = helm.Grid.of(w)
    m = torch.as_tensor(w.m, device="cuda").clone().requires_grad_(True)

    def f(mm):
        return misfit(mm, G, w.omegas, d_obs, w.sources, w.receivers, 0.0, 0.0, "fp64", 1e-12)

    # phi is accurate to ~1e-13 relative, so central differences with step
    # 1e-6 carry an error of ~1e-7 phi
    scale = abs(float(f(m).item()))
    assert scale > 0
    assert torch.autograd.gradcheck(f, (m,), eps=1e-6, atol=1e-6 * scale + 1e-12, rtol=1e-5, fast_mode=False)


def test_pipelined_serving_equals_serial(helm):
    """Factoring the next batch while the current one is solved (two streams,
    two host threads) gives bitwise the results of the serial schedule."""
    from paper_2301_10762_amd import serving as SV

    def reqs():
        return [make_request(SV, helm, rid, *spec)[0] for rid, spec in enumerate(SPECS)]
    srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36, max_chains=3)
    ser = {r.rid: r for r in SV.run_stream(srv, reqs(), realtime=False)}
    be = SV.HelmBackend("fp32_ir", 1e-10, stream=torch.cuda.Stream(), solve_stream=torch.cuda.Stream())
    srv = SV.Server(be, 1 << 36, max_chains=3)
    print("pipelined serving", flush=True)
    pip = SV.run_stream(srv, reqs(), realtime=False, pipelined=True)
    assert sorted(r.rid for r in pip) == sorted(ser) and srv.batches >= 2
    for r in pip:
        assert max(i.max_relres for i in r.infos) <= 1e-10
        for x, y in zip(r.X, ser[r.rid].X):
            assert torch.equal(x, y), r.rid


def test_lane_runs_reuse_memory(helm):
    """Consecutive lane runs in one process reuse the memory of the runs
    before them.  torch keeps a block freed on a stream for that stream;
    lane k of every run uses the same pooled stream, so three more runs add
    less than one run's results to the reserved memory (with new streams
    every run they would add about three)."""
    from paper_2301_10762_amd import serving as SV

    def run():
        reqs = [make_request(SV, helm, rid, 101, 40 + rid, (10.0 + rid,), 48)[0] for rid in range(6)]
        srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36, max_chains=4)
        res = SV.run_lanes(srv, reqs, lanes=3, realtime=False)
        torch.cuda.synchronize()
        srv.close()
        assert all(max(i.max_relres for i in r.infos) <= 1e-10 for r in res)
        return sum(x.numel() * x.element_size() for r in res for x in r.X)

    print("lane runs: memory reuse", flush=True)
    nbytes = run()
    torch.cuda.synchronize()
    before = torch.cuda.memory_reserved()
    for _ in range(3):
        assert run() == nbytes
    torch.cuda.synchronize()
    growth = torch.cuda.memory_reserved() - before
    assert growth < nbytes, (growth, nbytes)


@pytest.mark.parametrize("lanes", [2, 3])
def test_lane_serving_equals_serial(helm, lanes):
    """Batches run side by side on lanes (one stream and host thread each)
    give bitwise the results of the serial schedule, with resident factors
    reused across lanes."""
    from paper_2301_10762_amd import serving as SV

    def reqs():
        out = [make_request(SV, helm, rid, *spec, key=("m", rid))[0] for rid, spec in enumerate(SPECS)]
        # the same models again: resident factors made by one lane serve another
        out += [make_request(SV, helm, 10 + rid, *spec, key=("m", rid))[0] for rid, spec in enumerate(SPECS)]
        return out
    srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36, max_chains=3)
    ser = {r.rid: r for r in SV.run_stream(srv, reqs(), realtime=False)}
    srv.close()
    srv = SV.Server(SV.HelmBackend("fp32_ir", 1e-10), 1 << 36, max_chains=3, resident=True)
    print(f"lane serving, {lanes} lanes", flush=True)
    got = SV.run_lanes(srv, reqs(), lanes=lanes, realtime=False)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in got) == sorted(ser) and srv.batches >= 2
    assert srv.inflight_bytes == 0 and not srv.inflight_keys
    for r in got:
        assert max(i.max_relres for i in r.infos) <= 1e-10
        for x, y in zip(r.X, ser[r.rid].X):
            assert torch.equal(x, y), r.rid
    srv.close()
