"""Pins of the oracle's full Hessian product, its P2 preconditioner and PCG.

* H mt against central differences of the oracle gradient (whose own pins are
  in test_oracle.py), with the regulariser included;
* symmetry of H, and H = H^(1) + Gamma when the data are the model's own
  (zero residual, so H^(2) vanishes);
* the Cholesky solve with Gamma against the closed-form eigen-decomposition
  of the Neumann difference Laplacian (orthonormal DCT-II in each direction);
* PCG against textbook properties: at most k iterations for k distinct
  eigenvalues, one iteration with the exact inverse as preconditioner, and
  the solution of a dense SPD system.
"""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle
from oracle import Grid
from paper_2301_10762_amd import inputs as I


def _fwi(n=13, seed=4, n_src=3, n_rec=5, ppws=(8.0, 12.0)):
    w = I.small_layered(n, seed, n_src, n_rec, ppws=ppws)
    g = Grid.of(w)
    d_obs = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    return w, g, d_obs


def hvp_fd_error(hvp=None, t=1e-5, alpha=1e-3, mu=1e-4):
    """Largest relative gap between H mt and the central difference of the
    gradient along mt, over two random directions."""
    hvp = hvp or oracle.hvp
    w, g, d_obs = _fwi()
    rng = np.random.default_rng(3)
    dirs = [rng.standard_normal(g.N) for _ in range(2)]
    H = hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, dirs, alpha, mu)
    worst = 0.0
    for a, mt in enumerate(dirs):
        _, gp = oracle.misfit_grad(g, w.m + t * mt, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
        _, gm = oracle.misfit_grad(g, w.m - t * mt, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
        fd = (gp - gm) / (2 * t)
        worst = max(worst, np.linalg.norm(fd - H[a]) / np.linalg.norm(fd))
    return worst


def test_hvp_matches_gradient_differences():
    assert hvp_fd_error() < 1e-7


def test_hvp_second_order_part_is_material():
    """The case above exercises H^(2): H differs from H^(1) by far more than
    the finite-difference error."""
    w, g, d_obs = _fwi()
    rng = np.random.default_rng(3)
    mt = rng.standard_normal(g.N)
    H = oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, [mt])[0]
    H1 = oracle.gn_hvp(g, w.m, w.omegas, w.sources, w.receivers, [mt])[0][0]
    assert np.linalg.norm(H - H1) > 0.05 * np.linalg.norm(H)


def test_hvp_symmetric():
    w, g, d_obs = _fwi(n=11, seed=7)
    rng = np.random.default_rng(5)
    d1, d2 = rng.standard_normal(g.N), rng.standard_normal(g.N)
    h1, h2 = oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, [d1, d2], alpha=0.2, mu=0.01)
    assert abs(d2 @ h1 - d1 @ h2) <= 1e-11 * abs(d2 @ h1)


def test_hvp_is_gauss_newton_at_zero_residual():
    w = I.small_layered(11, 2, 3, 6, ppws=(9.0, 13.0))
    g = Grid.of(w)
    d_own = oracle.synth_data(g, w.m, w.omegas, w.sources, w.receivers)
    rng = np.random.default_rng(2)
    dirs = [rng.standard_normal(g.N) for _ in range(2)]
    H = oracle.hvp(g, w.m, w.omegas, d_own, w.sources, w.receivers, dirs, alpha=0.3, mu=0.02)
    _, Hgn = oracle.gn_hvp(g, w.m, w.omegas, w.sources, w.receivers, dirs, alpha=0.3, mu=0.02)
    assert np.linalg.norm(H - Hgn) <= 1e-12 * np.linalg.norm(Hgn)


def _dct_eigen(nx, nz, alpha, mu):
    """Eigenvalues of Gamma(alpha, mu) on the orthonormal DCT-II basis: the
    Neumann difference Laplacian of size n has eigenvalues 2 - 2 cos(pi k / n)
    and D_n^T D_n = (n - 1)^2 times it."""
    lx = (nx - 1) ** 2 * (2 - 2 * np.cos(np.pi * np.arange(nx) / nx))
    lz = (nz - 1) ** 2 * (2 - 2 * np.cos(np.pi * np.arange(nz) / nz))
    return alpha * (lz[:, None] + lx[None, :]) + mu


@pytest.mark.parametrize("nx,nz,alpha,mu", [(7, 5, 0.3, 0.05), (9, 12, 10.0, 1e-8), (16, 3, 1.0, 1.0)])
def test_gamma_solve_matches_dct_closed_form(nx, nz, alpha, mu):
    g = Grid(nx, nz, 1.0 / (nx - 1), 1.0 / (nz - 1))
    rng = np.random.default_rng(nx * nz)
    Y = rng.standard_normal((3, g.N))
    X = oracle.gamma_solve(g, alpha, mu, Y)
    lam = _dct_eigen(nx, nz, alpha, mu)
    # forward error of a backward-stable solve: a small multiple of kappa * eps
    tol = max(1e-12, 4 * np.finfo(float).eps * lam.max() / lam.min())
    for y, x in zip(Y, X):
        Yh = sfft.dctn(y.reshape(nz, nx), type=2, norm="ortho")
        xc = sfft.idctn(Yh / lam, type=2, norm="ortho").reshape(-1)
        assert np.linalg.norm(x - xc) <= tol * np.linalg.norm(xc)
    # and the eigenvalues are those of the regulariser matrix itself
    ev = np.sort(np.linalg.eigvalsh(oracle.regulariser(g, alpha, mu).toarray()))
    assert np.allclose(ev, np.sort(lam.reshape(-1)), rtol=1e-10, atol=1e-10 * ev.max())


def test_pcg_terminates_in_k_steps_for_k_eigenvalues():
    rng = np.random.default_rng(0)
    vals = np.array([1.0, 3.0, 7.0, 20.0])
    d = vals[rng.integers(0, 4, 40)]
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    A = Q @ np.diag(d) @ Q.T
    b = rng.standard_normal(40)
    x, it, hist = oracle.pcg(lambda v: A @ v, b, rtol=1e-10)
    assert it <= 4 + 1 and hist[-1] <= 1e-10
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(x)


def test_pcg_exact_preconditioner_one_step():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((30, 30))
    A = B @ B.T + 30 * np.eye(30)
    Ai = np.linalg.inv(A)
    b = rng.standard_normal(30)
    x, it, _ = oracle.pcg(lambda v: A @ v, b, lambda r: Ai @ r, rtol=1e-12)
    assert it == 1
    assert np.linalg.norm(x - Ai @ b) <= 1e-11 * np.linalg.norm(x)


def test_pcg_jacobi_dense_system():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((50, 50))
    A = B @ B.T + np.diag(np.linspace(1, 100, 50))
    b = rng.standard_normal(50)
    dg = np.diag(A).copy()
    x, it, hist = oracle.pcg(lambda v: A @ v, b, lambda r: r / dg, rtol=1e-12)
    assert hist[-1] <= 1e-12 and it <= 50 + 10
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(x)


def test_pcg_on_hessian_system_with_p2():
    """H rho = m' - m with the P2 = Gamma(alpha0, mu) preconditioner: the
    recurrence residual reaches the tolerance and the true residual follows."""
    w, g, d_obs = _fwi(n=11, seed=7)
    alpha, mu = 0.05, 1e-3

    def H(x):
        return oracle.hvp(g, w.m, w.omegas, d_obs, w.sources, w.receivers, [x], alpha, mu)[0]
    b = w.m_true - w.m
    x, it, hist = oracle.pcg(H, b, lambda r: oracle.gamma_solve(g, alpha, mu, r), rtol=1e-8)
    x_plain, it_plain, _ = oracle.pcg(H, b, rtol=1e-8)
    assert hist[-1] <= 1e-8
    r0 = np.linalg.norm(b - H(np.ones(g.N)))
    assert np.linalg.norm(b - H(x)) <= 1e-6 * r0
    assert np.linalg.norm(x - x_plain) <= 1e-5 * np.linalg.norm(x)
    assert it < it_plain
