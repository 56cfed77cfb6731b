"""GPU parity of the sliding-cubic restriction and the upper-level
derivatives (through the C ABI) against the FP64 oracle.

Tolerances: the restriction is a 16-term weighted sum computed in the same
FP64 arithmetic on both sides (1e-13 relative); phi, grad phi, H mt and the
upper-level derivatives follow from solves with relative residual <= 1e-10,
as for the gradient (1e-8); the whole chain through PCG to rtol 1e-12
against the oracle's dense Hessian solve, 1e-7.
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


def _points(g, n, seed, margin=0.0):
    rng = np.random.default_rng(seed)
    X, Z = (g.nx - 1) * g.hx, (g.nz - 1) * g.hz
    p = np.column_stack([rng.uniform(margin * X, (1 - margin) * X, n), rng.uniform(margin * Z, (1 - margin) * Z, n)])
    return p


@pytest.mark.parametrize("nx,nz", [(23, 17), (4, 4), (40, 9)])
def test_restrict_matches_oracle(helm, nx, nz):
    print(f"restrict {nx}x{nz}", flush=True)
    g = oracle.Grid(nx, nz, 0.025, 0.03)
    P = _points(g, 13, nx * nz)
    P[0] = [0.0, 0.0]
    P[1] = [(nx - 1) * g.hx, (nz - 1) * g.hz]
    P[2] = [3 * g.hx if nx > 3 else 0.0, 2 * g.hz]        # on a node
    rng = np.random.default_rng(1)
    U = rng.standard_normal((3, g.N)) + 1j * rng.standard_normal((3, g.N))
    S = oracle.Sensors(g, P)
    G = helm.Grid(nx, nz, g.hx, g.hz)
    for deriv in (0, 1, 2):
        out = helm.restrict(G, P, U, deriv).cpu().numpy()
        ref = (S.matrix(deriv) @ U.T).T
        assert_cols(out, ref, 1e-13, what=f"restriction, derivative {deriv}")


def test_restrict_rejects_outside_points(helm):
    G = helm.Grid(10, 10, 0.1, 0.1)
    with pytest.raises(helm.HelmError):
        helm.restrict(G, [[0.5, 0.95]], np.ones(100, dtype=np.complex128))
    with pytest.raises(helm.HelmError):
        helm.restrict(helm.Grid(3, 10, 0.1, 0.1), [[0.1, 0.1]], np.ones(30, dtype=np.complex128))


def _problem(n=25, seed=6, n_src=3, n_sens=5, ppws=(9.0, 13.0)):
    w = I.small_layered(n, seed, n_src, 4, ppws=ppws, n_dirs=2)
    g = oracle.Grid.of(w)
    # sensors between nodes, away from the sources at depth 2
    P = _points(g, n_sens, seed + 1, margin=0.05)
    P[:, 1] = np.clip(P[:, 1], 4.3 * g.hz, None)
    return w, g, P


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_context_at_points_matches_oracle(helm, precision):
    print(f"context at points {precision}", flush=True)
    w, g, P = _problem()
    S = oracle.Sensors(g, P)
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, S)
    phi_o, grad_o = oracle.misfit_grad(g, w.m, w.omegas, d, w.sources, S, 1e-3, 1e-5)
    Ho = oracle.hvp(g, w.m, w.omegas, d, w.sources, S, w.directions, 1e-3, 1e-5)
    Hc = helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, P, d, 1e-3, 1e-5, precision=precision,
                      tol=1e-10, with_grad=True)
    try:
        hv, _ = Hc.apply(np.array(w.directions))
        assert abs(Hc.phi - phi_o) <= 1e-9 * phi_o
        assert rel(Hc.grad.cpu().numpy(), grad_o) < 1e-8
        assert_cols(hv.cpu().numpy(), np.asarray(Ho), 1e-8, what="H m~ per direction")
    finally:
        Hc.close()


def test_upper_grad_matches_oracle(helm):
    """Same m_FWI stand-in, training model, sensors and rho on both sides."""
    print("upper_grad parity", flush=True)
    w, g, P = _problem()
    S = oracle.Sensors(g, P)
    m_fwi = w.m_true + 0.2 * (w.m - w.m_true)
    rng = np.random.default_rng(3)
    rho = np.asarray(w.directions[0]) + 0.1 * rng.standard_normal(g.N) * np.abs(w.directions[0]).max()
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, S)
    dd = np.zeros((len(w.omegas), len(w.sources), len(P), 2), dtype=np.complex128)
    for iw, om in enumerate(w.omegas):
        F = oracle.Factor(g, w.m_true, om)
        Ut = F.solve(oracle.unit_sources(g, w.sources))
        F.close()
        dd[iw, :, :, 0] = (S.matrix(1) @ Ut.T).T
        dd[iw, :, :, 1] = (S.matrix(2) @ Ut.T).T
    dp_o, da_o = oracle.upper_grad(g, m_fwi, w.m_true, w.omegas, w.sources, S, rho)
    Hc = helm.Hessian(helm.Grid.of(w), m_fwi, w.omegas, w.sources, P, d, 1e-3, 1e-5, tol=1e-10)
    try:
        dp, da, info = Hc.upper_grad(rho, dd)
    finally:
        Hc.close()
    assert rel(dp, dp_o) < 1e-8
    assert abs(da - da_o) <= 1e-10 * abs(da_o)
    assert info.solves >= len(w.omegas) * len(w.sources)


def test_upper_chain_on_gpu_matches_oracle(helm):
    """The whole chain on the GPU (training wavefield, data and its
    derivative through helm_restrict, the context, PCG for rho, the
    derivatives) against the oracle with a dense Hessian solve."""
    print("upper chain", flush=True)
    w, g, P = _problem(n=13, seed=2, n_src=2, n_sens=3, ppws=(7.0,))
    S = oracle.Sensors(g, P)
    alpha, mu = 1e-3, 1e-3
    m_fwi = w.m_true + 0.1 * (w.m - w.m_true)
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, S)
    H = oracle.hvp(g, m_fwi, w.omegas, d, w.sources, S, list(np.eye(g.N)), alpha, mu)
    rho_o = np.linalg.solve(H, w.m_true - m_fwi)
    dp_o, da_o = oracle.upper_grad(g, m_fwi, w.m_true, w.omegas, w.sources, S, rho_o)

    G = helm.Grid.of(w)
    E = I.point_sources(G.N, w.sources)
    Ft = [helm.factor(G, w.m_true, om, "fp64") for om in w.omegas]
    Ut = [F.solve(E, tol=1e-12)[0] for F in Ft]
    for F in Ft:
        F.close()
    dg = torch.stack([helm.restrict(G, P, U, 0) for U in Ut])
    ddg = torch.stack([torch.stack([helm.restrict(G, P, U, 1), helm.restrict(G, P, U, 2)], dim=-1) for U in Ut])
    Hc = helm.Hessian(G, m_fwi, w.omegas, w.sources, P, dg, alpha, mu, tol=1e-12)
    try:
        rho, it, rr, _ = Hc.pcg(w.m_true - m_fwi, prec_alpha=alpha, prec_mu=mu, rtol=1e-12)
        dp, da, _ = Hc.upper_grad(rho, ddg)
    finally:
        Hc.close()
    assert rel(rho.cpu().numpy(), rho_o) < 1e-7
    assert rel(dp, dp_o) < 1e-7
    assert abs(da - da_o) <= 1e-7 * abs(da_o)


@pytest.mark.slow
def test_upper_grad_201(helm):
    """201^2, four frequencies, 32 sources, 40 sensors between nodes: the
    derivatives for a given rho against the oracle."""
    print("upper_grad 201^2", flush=True)
    w = I.config_c4()
    g = oracle.Grid.of(w)
    rng = np.random.default_rng(11)
    X = (g.nx - 1) * g.hx
    P = np.column_stack([rng.uniform(0.02 * X, 0.98 * X, 40), rng.uniform(0.3 * X, 0.9 * X, 40)])
    S = oracle.Sensors(g, P)
    m_fwi = w.m_true + 0.1 * (w.m - w.m_true)
    rho = np.asarray(w.directions[1])
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, S)
    G = helm.Grid.of(w)
    E = I.point_sources(G.N, w.sources)
    ddg = []
    for om in w.omegas:
        F = helm.factor(G, w.m_true, om, "fp64")
        U = F.solve(E, tol=1e-12)[0]
        F.close()
        ddg.append(torch.stack([helm.restrict(G, P, U, 1), helm.restrict(G, P, U, 2)], dim=-1))
    ddg = torch.stack(ddg)
    Hc = helm.Hessian(G, m_fwi, w.omegas, w.sources, P, d, 1e-4, 1e-8, precision="fp32_ir", tol=1e-10)
    try:
        dp, da, _ = Hc.upper_grad(rho, ddg)
    finally:
        Hc.close()
    dp_o, da_o = oracle.upper_grad(g, m_fwi, w.m_true, w.omegas, w.sources, S, rho)
    assert rel(dp, dp_o) < 1e-8
    assert abs(da - da_o) <= 1e-10 * abs(da_o)
