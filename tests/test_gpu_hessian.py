"""GPU parity of the full Hessian product, the P2 preconditioner and PCG
(through the C ABI) against the FP64 oracle.

Tolerances:
  * H mt: the same FP64 arithmetic as the gradient, each product being two
    more solves whose relative residual is <= 1e-10, so 1e-8 as for the
    gradient;
  * P2^{-1} y: both sides are backward-stable solves with Gamma (Cholesky on
    the CPU, an orthogonal transform on the GPU), so their forward errors
    are bounded by a small multiple of kappa(Gamma) * eps; the bound used is
    max(1e-12, kappa * eps) with kappa from the closed-form eigenvalues;
  * PCG: the iterates of two CG runs that apply the same operators with
    errors of ~1e-10 agree to well within the stopping tolerance; the
    iteration counts may differ by one at the threshold.
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


def _kappa(nx, nz, alpha, mu):
    lx = (nx - 1) ** 2 * 4 * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2
    lz = (nz - 1) ** 2 * 4 * np.sin(np.pi * np.arange(nz) / (2 * nz)) ** 2
    ev = alpha * (lz[:, None] + lx[None, :]) + mu
    return ev.max() / ev.min()


# ------------------------------------------------------------------- P2 --

@pytest.mark.parametrize("nx,nz,alpha,mu", [(7, 5, 1.0, 1e-8), (33, 33, 10.0, 1e-8), (37, 29, 0.5, 1e-3),
                                            (65, 70, 2.0, 0.1), (2, 2, 0.0, 3.0)])
def test_gamma_solve_matches_oracle(helm, nx, nz, alpha, mu):
    print(f"gamma_solve {nx}x{nz} alpha={alpha} mu={mu}", flush=True)
    g = oracle.Grid(nx, nz, 1.0 / (nx - 1), 1.0 / (nz - 1))
    rng = np.random.default_rng(nx + 100 * nz)
    Y = rng.standard_normal((3, g.N))
    Xo = oracle.gamma_solve(g, alpha, mu, Y)
    X = helm.gamma_solve(helm.Grid(nx, nz, g.hx, g.hz), alpha, mu, Y).cpu().numpy()
    tol = max(1e-12, np.finfo(float).eps * _kappa(nx, nz, alpha, mu))
    for a in range(3):
        assert rel(X[a], Xo[a]) <= tol, (a, rel(X[a], Xo[a]), tol)


def test_gamma_solve_in_place_and_401_residual(helm):
    """At 401^2 (the size of the largest configuration): Gamma x = y to the
    backward error of an orthogonal-transform solve, X overwriting Y."""
    print("gamma_solve 401x401 in place", flush=True)
    n = 401
    g = oracle.Grid(n, n, 1.0 / (n - 1), 1.0 / (n - 1))
    alpha, mu = 10.0, 1e-2
    rng = np.random.default_rng(7)
    y = rng.standard_normal(g.N)
    Yd = torch.as_tensor(y, device="cuda").reshape(1, -1).clone()
    L = helm.lib()
    import ctypes
    helm._check(L.helm_gamma_solve(ctypes.byref(helm.Grid(n, n, g.hx, g.hx).c()), alpha, mu, 1,
                                   helm._ptr(Yd), helm._ptr(Yd), None))
    x = Yd.cpu().numpy()[0]
    G = oracle.regulariser(g, alpha, mu)
    lam_max = alpha * 8 * (n - 1) ** 2 + mu
    assert np.linalg.norm(G @ x - y) <= 64 * np.finfo(float).eps * lam_max * np.linalg.norm(x)


def test_gamma_solve_rejects_singular(helm):
    g = helm.Grid(9, 9, 0.1, 0.1)
    with pytest.raises(helm.HelmError):
        helm.gamma_solve(g, 1.0, 0.0, np.ones(81))


# --------------------------------------------------------- Hessian products --

def _fwi(w):
    g = oracle.Grid.of(w)
    return g, oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_full_hessian_matches_oracle(helm, precision):
    print(f"full Hessian 29x29 {precision}", flush=True)
    w = I.small_layered(29, 13, 4, 7, ppws=(9.0, 14.0), n_dirs=3)
    g, d_obs = _fwi(w)
    alpha, mu = 1e-3, 1e-6
    Ho = oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, w.directions, alpha, mu)
    phi_o, grad_o = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
    Hc = helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, w.receivers, d_obs, alpha, mu,
                      precision=precision, tol=1e-10, with_grad=True)
    try:
        hv, info = Hc.apply(np.array(w.directions))
        hv = hv.cpu().numpy()
        for a in range(len(w.directions)):
            assert rel(hv[a], Ho[a]) < 1e-8, (a, rel(hv[a], Ho[a]))
        assert abs(Hc.phi - phi_o) <= 1e-9 * phi_o
        assert rel(Hc.grad.cpu().numpy(), grad_o) < 1e-8
        # v and z solves per frequency, source and direction
        S, D = len(w.sources), len(w.directions)
        assert info.solves >= len(w.omegas) * 2 * S * D
        assert info.max_relres <= 1e-10
        # a second product on the same context gives the same result
        hv2, _ = Hc.apply(np.array(w.directions))
        assert np.array_equal(hv2.cpu().numpy(), hv)
    finally:
        Hc.close()


def test_full_hessian_ragged_grid_single_direction(helm):
    """A grid whose row length is not a multiple of the 16-wide tiles, one
    source, one frequency, one direction (the degenerate counts)."""
    print("full Hessian 37x23 single", flush=True)
    w = I.small_layered(37, 5, 1, 3, ppws=(11.0,), n_dirs=1)
    # a non-square grid: keep the first 23 rows of the 37 x 37 model
    nz = 23
    g = oracle.Grid(37, nz, w.hx, w.hz)
    m = w.m[: 37 * nz]
    m_true = w.m_true[: 37 * nz]
    mt = np.asarray(w.directions[0])[: 37 * nz]
    d_obs = oracle.synth_data(g, m_true, w.omegas, w.sources, w.receivers)
    Ho = oracle.hvp(g, m, w.omegas, d_obs, w.sources, w.receivers, [mt], 0.0, 0.0)
    Hc = helm.Hessian(helm.Grid(37, nz, w.hx, w.hz), m, w.omegas, w.sources, w.receivers, d_obs, tol=1e-10)
    try:
        hv, _ = Hc.apply(mt)
        assert rel(hv.cpu().numpy()[0], Ho[0]) < 1e-8
    finally:
        Hc.close()


def test_hessian_repeated_receivers(helm):
    """Receivers listed twice count twice in R^* R (and in R^* eps)."""
    print("full Hessian repeated receivers", flush=True)
    w = I.small_layered(21, 9, 2, 4, ppws=(10.0,), n_dirs=2)
    rec = [int(w.receivers[0]), int(w.receivers[2]), int(w.receivers[2]), int(w.receivers[3]),
           int(w.receivers[0]), int(w.receivers[2])]
    g = oracle.Grid.of(w)
    d_obs = oracle.synth_data(g, w.m_true, w.omegas, w.sources, rec)
    Ho = oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, rec, w.directions, 0.01, 0.001)
    Hgo = oracle.gn_hvp(g, w.m, w.omegas, w.sources, rec, w.directions, 0.01, 0.001)[1]
    G = helm.Grid.of(w)
    Hf = helm.Hessian(G, w.m, w.omegas, w.sources, rec, d_obs, 0.01, 0.001, tol=1e-10)
    Hg = helm.Hessian(G, w.m, w.omegas, w.sources, rec, None, 0.01, 0.001, tol=1e-10)
    try:
        a, _ = Hf.apply(np.array(w.directions))
        b, _ = Hg.apply(np.array(w.directions))
        assert rel(a.cpu().numpy(), Ho) < 1e-8
        assert rel(b.cpu().numpy(), Hgo) < 1e-8
    finally:
        Hf.close()
        Hg.close()


def test_full_equals_gauss_newton_at_zero_residual(helm):
    print("full vs GN at zero residual", flush=True)
    w = I.small_layered(31, 3, 3, 6, ppws=(10.0, 13.0), n_dirs=2)
    g = oracle.Grid.of(w)
    d_own = oracle.synth_data(g, w.m, w.omegas, w.sources, w.receivers)
    G = helm.Grid.of(w)
    Hf = helm.Hessian(G, w.m, w.omegas, w.sources, w.receivers, d_own, 0.2, 0.01, tol=1e-10)
    Hg = helm.Hessian(G, w.m, w.omegas, w.sources, w.receivers, None, 0.2, 0.01, tol=1e-10)
    try:
        a, _ = Hf.apply(np.array(w.directions))
        b, _ = Hg.apply(np.array(w.directions))
        assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-9
    finally:
        Hf.close()
        Hg.close()


@pytest.mark.slow
def test_full_hessian_c4_size(helm):
    """201^2, 4 frequencies, 32 sources, 8 directions in one product (the
    benchmark's launch configuration): direction 0 against the oracle, and
    the symmetry of H over all pairs of directions."""
    print("full Hessian 201^2 x 8 directions", flush=True)
    w = I.config_c4()
    g, d_obs = _fwi(w)
    alpha, mu = 1e-3, 1e-6
    Hc = helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, w.receivers, d_obs, alpha, mu,
                      precision="fp32_ir", tol=1e-10)
    try:
        D = np.array(w.directions)
        hv, info = Hc.apply(D)
        hv = hv.cpu().numpy()
    finally:
        Hc.close()
    assert info.max_relres <= 1e-10
    M = D @ hv.T
    assert np.max(np.abs(M - M.T)) <= 1e-8 * np.max(np.abs(M))
    Ho = oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, [D[0]], alpha, mu)
    assert rel(hv[0], Ho[0]) < 1e-8


# -------------------------------------------------------------------- PCG --

@pytest.mark.parametrize("use_p2", [True, False])
def test_pcg_matches_oracle(helm, use_p2):
    print(f"pcg 15x15 p2={use_p2}", flush=True)
    w = I.small_layered(15, 7, 3, 5, ppws=(8.0, 12.0))
    g, d_obs = _fwi(w)
    alpha, mu = 0.05, 1e-3
    b = w.m_true - w.m

    def H(x):
        return oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, [x], alpha, mu)[0]
    pinv = (lambda r: oracle.gamma_solve(g, alpha, mu, r)) if use_p2 else None
    xo, it_o, hist = oracle.pcg(H, b, pinv, rtol=1e-9)
    Hc = helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, w.receivers, d_obs, alpha, mu, tol=1e-11)
    try:
        x, it, rr, info = Hc.pcg(b, prec_alpha=alpha if use_p2 else 0.0, prec_mu=mu if use_p2 else 0.0, rtol=1e-9)
    finally:
        Hc.close()
    assert rr <= 1e-9
    assert abs(it - it_o) <= 1, (it, it_o)
    assert rel(x.cpu().numpy(), xo) < 1e-6
    assert info.solves >= (it + 1) * len(w.omegas) * 2 * len(w.sources)


def test_pcg_reports_nonconvergence(helm):
    print("pcg maxit", flush=True)
    w = I.small_layered(15, 7, 3, 5, ppws=(8.0,))
    g, d_obs = _fwi(w)
    Hc = helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, w.receivers, d_obs, 0.05, 1e-3, tol=1e-11)
    try:
        with pytest.raises(helm.HelmError) as e:
            Hc.pcg(w.m_true - w.m, rtol=1e-14, maxit=2)
        assert e.value.code == helm.ENOCONV
    finally:
        Hc.close()


def test_pcg_batch_equals_single(helm):
    """Three systems (different models and grids) in lockstep: each follows
    exactly the iteration it follows alone (bitwise), whatever the others."""
    print("pcg batch", flush=True)
    cases = []
    for n, seed in ((15, 7), (17, 3), (15, 11)):
        w = I.small_layered(n, seed, 3, 5, ppws=(8.0, 12.0))
        g, d_obs = _fwi(w)
        cases.append((w, d_obs))
    alpha, mu = 0.05, 1e-3
    ctx = [helm.Hessian(helm.Grid.of(w), w.m, w.omegas, w.sources, w.receivers, d, alpha, mu, tol=1e-11)
           for w, d in cases]
    try:
        bs = [w.m_true - w.m for w, _ in cases]
        xs, its, rrs, sts, _ = helm.pcg_batch(ctx, bs, prec_alpha=alpha, prec_mu=mu, rtol=1e-9)
        for c, H in enumerate(ctx):
            x1, it1, rr1, _ = H.pcg(bs[c], prec_alpha=alpha, prec_mu=mu, rtol=1e-9)
            assert sts[c] == "converged"
            assert its[c] == it1 and rrs[c] == rr1
            assert torch.equal(xs[c], x1)
    finally:
        for H in ctx:
            H.close()


@pytest.mark.slow
def test_pcg_c4_size_true_residual(helm):
    """The benchmark's Hessian system (201^2, 4 frequencies, 32 sources, P2,
    rtol 1e-6, FP64 context): the oracle's own product with the returned rho
    leaves a residual within the tolerance."""
    print("pcg 201^2 true residual", flush=True)
    w = I.config_c4()
    g = oracle.Grid.of(w)
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    m_fwi = w.m_true + 0.1 * (w.m - w.m_true)
    b = w.m_true - m_fwi
    alpha, mu = 1e-4, 1e-8
    Hc = helm.Hessian(helm.Grid.of(w), m_fwi, w.omegas, w.sources, w.receivers, d, alpha, mu, tol=1e-10)
    try:
        rho, it, rr, _ = Hc.pcg(b, prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=300)
    finally:
        Hc.close()
    rho = rho.cpu().numpy()
    H = lambda x: oracle.hvp(g, m_fwi, w.omegas, d, w.sources, w.receivers, [x], alpha, mu)[0]
    r0 = np.linalg.norm(b - H(np.ones(g.N)))
    assert rr <= 1e-6
    assert np.linalg.norm(b - H(rho)) <= 2e-6 * r0
