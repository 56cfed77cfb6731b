"""GPU parity of point sources between nodes, h_x != h_z and data from a
second grid (the inverse-crime-free workflow) against the FP64 oracle.

Tolerances: the loads are the same four products on both sides (1e-15);
phi, grad, H mt and data follow from solves with relative residual <= 1e-10
(1e-8); FWI histories as in the FWI parity tests (1e-9).
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


def _pts(g, n, seed, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    rng = np.random.default_rng(seed)
    X, Z = (g.nx - 1) * g.hx, (g.nz - 1) * g.hz
    return np.column_stack([rng.uniform(lo[0] * X, hi[0] * X, n), rng.uniform(lo[1] * Z, hi[1] * Z, n)])


@pytest.mark.parametrize("nx,nz,hx,hz", [(17, 11, 0.03, 0.02), (2, 2, 1.0, 0.5), (40, 33, 0.025, 0.025)])
def test_point_sources_match_oracle(helm, nx, nz, hx, hz):
    print(f"point sources {nx}x{nz}", flush=True)
    g = oracle.Grid(nx, nz, hx, hz)
    P = _pts(g, 9, nx)
    P[0] = [0.0, 0.0]
    P[1] = [(nx - 1) * hx, (nz - 1) * hz]
    P[2] = [(nx - 1) * hx, 0.0]
    B = helm.point_sources(helm.Grid(nx, nz, hx, hz), P).cpu().numpy()
    assert np.max(np.abs(B - oracle.point_sources(g, P))) <= 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_context_point_sources_unequal_spacing(helm, precision):
    """phi, grad and H mt with point sources, sensors at points and
    h_x != h_z."""
    print(f"context point sources {precision}", flush=True)
    w = I.small_layered(23, 9, 3, 4, ppws=(9.0, 12.0), n_dirs=2)
    g = oracle.Grid(w.nx, w.nz, w.hx, 0.7 * w.hz)
    src = _pts(g, 3, 1, (0.1, 0.05), (0.9, 0.2))
    P = _pts(g, 5, 2, (0.05, 0.4), (0.95, 0.95))
    S = oracle.Sensors(g, P)
    d = oracle.synth_data(g, w.m_true, w.omegas, src, S)
    phi_o, grad_o = oracle.misfit_grad(g, w.m, w.omegas, d, src, S, 1e-3, 1e-5)
    Ho = oracle.hvp(g, w.m, w.omegas, d, src, S, w.directions, 1e-3, 1e-5)
    G = helm.Grid(g.nx, g.nz, g.hx, g.hz)
    Hc = helm.Hessian(G, w.m, w.omegas, src, P, d, 1e-3, 1e-5, precision=precision, tol=1e-10, with_grad=True)
    try:
        hv, _ = Hc.apply(np.array(w.directions))
        assert abs(Hc.phi - phi_o) <= 1e-9 * phi_o
        assert rel(Hc.grad.cpu().numpy(), grad_o) < 1e-8
        assert_cols(hv.cpu().numpy(), np.asarray(Ho), 1e-8, what="H m~ per direction")
    finally:
        Hc.close()


def test_misfit_gradient_unequal_spacing_nodes(helm):
    print("misfit hx != hz", flush=True)
    w = I.small_layered(19, 3, 3, 6, ppws=(10.0,))
    g = oracle.Grid(w.nx, w.nz, 1.3 * w.hx, w.hz)
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    phi_o, grad_o = oracle.misfit_grad(g, w.m, w.omegas, d, w.sources, w.receivers)
    phi, grad, _ = helm.misfit_grad(helm.Grid(g.nx, g.nz, g.hx, g.hz), w.m, w.omegas, d, w.sources, w.receivers,
                                    tol=1e-10)
    assert abs(phi - phi_o) <= 1e-10 * phi_o
    assert rel(grad.cpu().numpy(), grad_o) < 1e-8


def test_data_from_second_grid_and_fwi(helm):
    """The inverse-crime-free workflow: the training data come from a finer,
    non-nested grid (the model resampled onto it; the sources and sensors,
    nodes of the inversion grid, fall between its nodes); FWI then runs on
    the inversion grid.  The GPU computes the data (point sources, solves,
    helm_restrict) and the FWI; the oracle does the same on the CPU."""
    print("second-grid data + fwi", flush=True)
    w = I.small_layered(21, 4, 3, 8, ppws=(8.0, 12.0))
    g = oracle.Grid.of(w)
    X = (g.nx - 1) * g.hx
    nf = 31
    gf = oracle.Grid(nf, nf, X / (nf - 1), X / (nf - 1))
    m_fine = I.resample(w.m_true, (g.nx, g.nz, g.hx, g.hz), (gf.nx, gf.nz, gf.hx, gf.hz))
    src = np.array([[(k % g.nx) * g.hx, (k // g.nx) * g.hz] for k in w.sources])
    P = np.array([[(k % g.nx) * g.hx, (k // g.nx) * g.hz] for k in w.receivers])
    Sf = oracle.Sensors(gf, P)
    d_o = oracle.synth_data(gf, m_fine, w.omegas, src, Sf)
    # the same data on the GPU
    Gf = helm.Grid(gf.nx, gf.nz, gf.hx, gf.hz)
    B = helm.point_sources(Gf, src)
    d_g = []
    for om in w.omegas:
        F = helm.factor(Gf, m_fine, om, "fp64")
        U, _ = F.solve(B, tol=1e-12)
        F.close()
        d_g.append(helm.restrict(Gf, P, U, 0))
    d_g = torch.stack(d_g)
    assert_cols(d_g.cpu().numpy().reshape(-1, d_o.shape[-1]), d_o.reshape(-1, d_o.shape[-1]), 1e-10,
                what="second-grid data per (frequency, source)")
    # FWI on the inversion grid with these data
    kw = dict(memory=4, max_iters=6, gtol=1e-8)
    mo, oinfo = oracle.fwi(g, w.m, w.omegas, d_o, w.sources, w.receivers, 1e-3, 1e-4, **kw)
    m, info = helm.fwi(helm.Grid.of(w), w.m, w.omegas, d_g, w.sources, w.receivers, 1e-3, 1e-4, tol=1e-11, **kw)
    assert info["iterations"] == oinfo["iterations"] and info["evals"] == oinfo["evals"]
    h, ho = np.array(info["history"]), np.array(oinfo["history"])
    assert np.max(np.abs(h - ho) / np.abs(ho)) <= 1e-9
    assert rel(m.cpu().numpy(), mo) <= 1e-8
