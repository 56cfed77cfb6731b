"""Pins of the FP64 CPU oracle against facts the paper and mathematics fix.

None of these compare the oracle with itself: the referees are an
independent P1 element assembly, a hand-derived golden stencil, LAPACK
(numpy/scipy) solves, manufactured solutions, the free-space Green's function,
reciprocity, Green's identity and finite differences.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla
import scipy.special

import oracle
from oracle import Grid
from paper_2301_10762_amd import inputs as I
from tests import fem_p1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- assembly --

def _split_operator(g, m):
    """S, d, b read back from the oracle: A(w=0) = S; A(w=1) - S = -d m - i b sqrt m."""
    S = oracle.matrix(g, m, 0.0).toarray()
    A1 = oracle.matrix(g, m, 1.0).toarray()
    D = np.diag(A1 - S)
    return S.real, -D.real / m, -D.imag / np.sqrt(m)


def test_golden_3x3_stencil(oracle_mod):
    """App. A.1 entries on a 3x3 grid with hx=2, hz=1, derived by hand."""
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "stencil_3x3_hx2_hz1.txt"))
             if ln.strip() and not ln.startswith("#")]
    diag_rows, off_rows, section = [], [], 0
    for ln in lines:
        if ln[0] == "k" and len(ln) == 4:
            section = 1
            continue
        if ln[0] == "k" and len(ln) == 3:
            section = 2
            continue
        (diag_rows if section == 1 else off_rows).append([float(x) for x in ln])
    g = Grid(3, 3, 2.0, 1.0)
    m = np.linspace(0.3, 1.1, 9)
    S, d, b = _split_operator(g, m)
    for k, skk, dk, bk in diag_rows:
        k = int(k)
        assert S[k, k] == pytest.approx(skk, abs=1e-14)
        assert d[k] == pytest.approx(dk, abs=1e-14)
        assert b[k] == pytest.approx(bk, abs=1e-14)
    expected_off = np.zeros((9, 9))
    for k, l, v in off_rows:
        expected_off[int(k), int(l)] = expected_off[int(l), int(k)] = v
    off = S - np.diag(np.diag(S))
    np.testing.assert_allclose(off, expected_off, atol=1e-14)


@pytest.mark.parametrize("nx,nz,hx,hz", [(5, 4, 0.7, 0.4), (6, 6, 0.1, 0.1), (4, 7, 0.3, 0.9)])
def test_operator_matches_p1_element_assembly(oracle_mod, nx, nz, hx, hz):
    """S equals the P1 stiffness for both triangulation directions (the
    five-point statement of App. A.1); d and b equal the nodal quadratures."""
    rng = np.random.default_rng(nx * 100 + nz)
    m = rng.uniform(0.2, 1.5, nx * nz)
    S, d, b = _split_operator(Grid(nx, nz, hx, hz), m)
    _, S1, S2, dref, bref = fem_p1.operator(nx, nz, hx, hz, m, 1.0)
    np.testing.assert_allclose(S, S1.toarray(), atol=1e-13)
    np.testing.assert_allclose(S, S2.toarray(), atol=1e-13)
    np.testing.assert_allclose(d, dref, rtol=1e-12)
    np.testing.assert_allclose(b, bref, rtol=1e-12, atol=1e-15)


def test_operator_is_complex_symmetric(oracle_mod):
    w = I.small_layered(9, 3, 2, 3)
    A = oracle.matrix(Grid.of(w), w.m, w.omegas[0])
    assert abs(A - A.T).max() == 0.0
    # and not Hermitian: the impedance term is imaginary
    assert abs(A - A.conj().T).max() > 0.0


# ------------------------------------------------------------------- solves --

def _dense_reference(nx, nz, hx, hz, m, w):
    A, *_ = fem_p1.operator(nx, nz, hx, hz, m, w)
    return A.toarray()


@pytest.mark.parametrize("nx,nz", [(7, 5), (4, 9), (11, 11)])
def test_solve_matches_dense_lapack(oracle_mod, nx, nz):
    rng = np.random.default_rng(nx + 7 * nz)
    hx, hz = 0.05, 0.04
    m = rng.uniform(0.1, 0.5, nx * nz)
    w = 25.0
    g = Grid(nx, nz, hx, hz)
    B = rng.standard_normal((3, g.N)) + 1j * rng.standard_normal((3, g.N))
    Ad = _dense_reference(nx, nz, hx, hz, m, w)
    F = oracle.Factor(g, m, w)
    X = F.solve(B)
    Xr = np.linalg.solve(Ad, B.T).T
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) < 1e-12
    L = F.adjoint_solve(B)
    Lr = np.linalg.solve(Ad.conj().T, B.T).T
    assert np.linalg.norm(L - Lr) / np.linalg.norm(Lr) < 1e-12


def test_solve_matches_lapack_banded_c1(oracle_mod):
    """Config of the 33 x 33 blob problem: zgbsv through scipy.linalg.solve_banded."""
    w = I.config_c1()
    g = Grid.of(w)
    A, *_ = fem_p1.operator(w.nx, w.nz, w.hx, w.hz, w.m, w.omegas[0])
    A = A.toarray()
    kl = ku = w.nx
    ab = np.zeros((kl + ku + 1, g.N), dtype=complex)
    for j in range(g.N):
        for i in range(max(0, j - ku), min(g.N, j + kl + 1)):
            ab[ku + i - j, j] = A[i, j]
    B = I.point_sources(g.N, w.sources)
    Xr = scipy.linalg.solve_banded((kl, ku), ab, B.T).T
    X = oracle.Factor(g, w.m, w.omegas[0]).solve(B)
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) < 1e-12


def test_discrete_manufactured_solution(oracle_mod):
    """b = A x* with A from the element assembly; x* recovered to rounding."""
    w = I.small_layered(41, 5, 1, 1, ppws=(8.0,))
    g = Grid.of(w)
    A, *_ = fem_p1.operator(w.nx, w.nz, w.hx, w.hz, w.m, w.omegas[0])
    rng = np.random.default_rng(3)
    xs = rng.standard_normal((2, g.N)) + 1j * rng.standard_normal((2, g.N))
    B = (A @ xs.T).T
    X = oracle.Factor(g, w.m, w.omegas[0]).solve(B)
    assert np.linalg.norm(X - xs) / np.linalg.norm(xs) < 1e-10


def test_solution_residual_small_at_201(oracle_mod):
    """Relative residual of the banded LU on a 201^2 layered problem at 10 PPW."""
    w = I.config_c2()
    g = Grid.of(w)
    F = oracle.Factor(g, w.m, w.omegas[-1])
    B = oracle.unit_sources(g, w.sources[:4])
    X = F.solve(B)
    assert oracle.relres(g, w.m, w.omegas[-1], X, B).max() < 1e-12
    L = F.adjoint_solve(B)
    assert oracle.relres(g, w.m, w.omegas[-1], L, B, adjoint=True).max() < 1e-12


# ----------------------------------------------------------- discretisation --

def _plane_wave_error(n, k, theta):
    """Manufactured plane wave u = exp(i k (x cos t + z sin t)) on the unit
    square, m = 1, f = 0, impedance data f_b = du/dn - i k u injected as the
    nodal boundary quadrature (App. A.1, (f_b)_k) edge by edge."""
    h = 1.0 / (n - 1)
    g = Grid(n, n, h, h)
    N = g.N
    x = (np.arange(N) % n) * h
    z = (np.arange(N) // n) * h
    kx, kz = k * math.cos(theta), k * math.sin(theta)
    u = np.exp(1j * (kx * x + kz * z))
    f = np.zeros(N, dtype=complex)
    for a, b, L, (nxv, nzv) in fem_p1.boundary_edges(n, n, h, h):
        for p in (a, b):
            dudn = 1j * (kx * nxv + kz * nzv) * u[p]
            f[p] += 0.5 * L * (dudn - 1j * k * u[p])
    uh = oracle.Factor(g, np.ones(N), k).solve(f)[0]
    return np.linalg.norm(uh - u) / np.linalg.norm(u)


def test_plane_wave_second_order(oracle_mod):
    """The impedance problem (eq (forward)) with a manufactured plane wave:
    error O(h^2), ratio ~4 per halving of h."""
    k = 2 * math.pi * 2.0
    errs = [_plane_wave_error(n, k, 0.3) for n in (33, 65, 129)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.6 < r2 < 4.4, errs
    assert errs[-1] < 5e-3


def _green_error(ppw, n=161):
    """Point source at the centre; compare with the outgoing free-space
    Green's function +(i/4) H0^(1)(k r) of -(Laplace + k^2) in the ring
    3h < r < one wavelength."""
    h = 1.0 / (n - 1)
    k = 2 * math.pi / (ppw * h)
    g = Grid(n, n, h, h)
    c = (n // 2) * n + n // 2
    u = oracle.Factor(g, np.ones(g.N), k).solve(oracle.unit_sources(g, [c]))[0]
    x = (np.arange(g.N) % n) * h - (n // 2) * h
    z = (np.arange(g.N) // n) * h - (n // 2) * h
    r = np.hypot(x, z)
    ring = (r > 3 * h) & (r < ppw * h)
    G = 0.25j * scipy.special.hankel1(0, k * r[ring])
    return np.linalg.norm(u[ring] - G) / np.linalg.norm(G), u, ring, r, k


def test_free_space_green_function(oracle_mod):
    """Discretisation-level agreement with +(i/4) H0^(1)(kr); the opposite
    sign (an incoming wave) is far off, which pins the impedance sign."""
    e10, u, ring, r, k = _green_error(10.0)
    e20, *_ = _green_error(20.0)
    assert e10 < 0.10 and e20 < 0.04 and e20 < e10, (e10, e20)
    wrong = -0.25j * scipy.special.hankel1(0, k * r[ring])
    assert np.linalg.norm(u[ring] - wrong) / np.linalg.norm(wrong) > 1.0


# --------------------------------------------------------------- identities --

def test_reciprocity(oracle_mod):
    """A = A^T  =>  u_s(x_r) = u_r(x_s)."""
    w = I.small_layered(31, 7, 5, 5)
    g = Grid.of(w)
    nodes = np.concatenate([w.sources, w.receivers])
    U = oracle.Factor(g, w.m, w.omegas[0]).solve(oracle.unit_sources(g, nodes))
    M = U[:, nodes]
    assert np.abs(M - M.T).max() / np.abs(M).max() < 1e-12


def test_green_identity_adjoint_consistency(oracle_mod):
    """(S f, g) = (f, S^* g) (eq (Green)) in discrete form, and
    A^{-*} g = conj(A^{-1} conj g) because A is complex symmetric."""
    w = I.small_layered(25, 9, 1, 1)
    g = Grid.of(w)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    q = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    F = oracle.Factor(g, w.m, w.omegas[0])
    Sf = F.solve(f)[0]
    Sq = F.adjoint_solve(q)[0]
    lhs = np.vdot(q, Sf)       # (S f, q) = sum Sf conj(q)
    rhs = np.vdot(Sq, f)       # (f, S^* q)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    alt = np.conj(F.solve(np.conj(q))[0])
    assert np.linalg.norm(alt - Sq) / np.linalg.norm(Sq) < 1e-12


def test_restriction_adjointness(oracle_mod):
    """<R u, z> = (u, R^* z) (eq (I1)), including a repeated receiver."""
    rng = np.random.default_rng(1)
    N = 50
    rec = np.array([3, 17, 17, 40])
    U = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    Z = rng.standard_normal((2, 4)) + 1j * rng.standard_normal((2, 4))
    lhs = np.sum(oracle.restrict(U, rec) * np.conj(Z))
    rhs = np.sum(U * np.conj(oracle.restrict_adjoint(Z, rec, N)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ----------------------------------------------------------------- gradient --

def _small_fwi(n=15, seed=4, n_src=3, n_rec=6, ppws=(8.0, 12.0)):
    w = I.small_layered(n, seed, n_src, n_rec, ppws=ppws)
    g = Grid.of(w)
    d_obs = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    return w, g, d_obs


def test_gradient_central_differences(oracle_mod):
    """dphi/dm along random unit directions vs central differences, t = 1e-6
    (Thm A.1 / App. B.1 formula, including the boundary term)."""
    w, g, d_obs = _small_fwi()
    alpha, mu = 1e-3, 1e-6
    phi, grad = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
    rng = np.random.default_rng(11)
    t = 1e-6
    for _ in range(8):
        dlt = rng.standard_normal(g.N)
        dlt /= np.linalg.norm(dlt)
        fp, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
        fm, _ = oracle.misfit_grad(g, w.m - t * dlt, w.omegas, d_obs, w.sources, w.receivers, alpha, mu)
        fd = (fp - fm) / (2 * t)
        an = grad @ dlt
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(grad)), (fd, an)


def test_gradient_boundary_only_direction(oracle_mod):
    """A direction supported on boundary nodes only exercises the
    b_k i w / (2 sqrt m_k) term of the gradient."""
    w, g, d_obs = _small_fwi(seed=6)
    phi, grad = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers)
    d, b = oracle.weights(g)
    dlt = np.where(b > 0, 1.0, 0.0)
    dlt /= np.linalg.norm(dlt)
    t = 1e-6
    fp, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d_obs, w.sources, w.receivers)
    fm, _ = oracle.misfit_grad(g, w.m - t * dlt, w.omegas, d_obs, w.sources, w.receivers)
    fd = (fp - fm) / (2 * t)
    assert abs(fd - grad @ dlt) <= 1e-6 * abs(fd)


def test_gradient_taylor_remainder_second_order(oracle_mod):
    w, g, d_obs = _small_fwi(seed=8)
    phi0, grad = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers)
    rng = np.random.default_rng(2)
    dlt = rng.standard_normal(g.N) * w.m * 0.05
    rem = []
    ts = [1.0, 0.5, 0.25]
    for t in ts:
        f, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d_obs, w.sources, w.receivers)
        rem.append(abs(f - phi0 - t * (grad @ dlt)))
    slopes = [math.log(rem[i] / rem[i + 1]) / math.log(2.0) for i in range(2)]
    assert all(1.8 < s < 2.2 for s in slopes), slopes


def test_solve_counts_two_per_source_frequency(oracle_mod):
    """Thm A.1: two Helmholtz solves per (s, w) for phi and grad phi."""
    w, g, d_obs = _small_fwi()
    _, _, fields = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers,
                                      return_fields=True)
    for _, _, solves in fields:
        assert solves == 2 * len(w.sources)


def test_zero_misfit_at_true_model(oracle_mod):
    w, g, d_obs = _small_fwi()
    phi, grad = oracle.misfit_grad(g, w.m_true, w.omegas, d_obs, w.sources, w.receivers)
    assert phi < 1e-25 and np.abs(grad).max() < 1e-12


# ------------------------------------------------------------ Gauss-Newton --

def _jacobian_fd(w, g, t=1e-6):
    """R du/dm_k for every k by central differences: complex [sum(Nr*S)] x N."""
    cols = []
    for k in range(g.N):
        e = np.zeros(g.N)
        e[k] = t
        blocks = []
        for om in w.omegas:
            Up = oracle.Factor(g, w.m + e, om).solve(oracle.unit_sources(g, w.sources))
            Um = oracle.Factor(g, w.m - e, om).solve(oracle.unit_sources(g, w.sources))
            blocks.append(((oracle.restrict(Up, w.receivers) - oracle.restrict(Um, w.receivers)) / (2 * t)).ravel())
        cols.append(np.concatenate(blocks))
    return np.array(cols).T


def test_gn_hessian_matches_jacobian(oracle_mod):
    """H^(1) = Re(J^* J) (eq (h1)) with J by central differences; the
    adjoint-state product of the lemma for H^(1) must reproduce it."""
    w = I.small_layered(7, 12, 2, 4, ppws=(6.0, 9.0))
    g = Grid.of(w)
    J = _jacobian_fd(w, g)
    H = np.real(J.conj().T @ J)
    rng = np.random.default_rng(5)
    dirs = [rng.standard_normal(g.N) for _ in range(3)]
    hv, hv_reg = oracle.gn_hvp(g, w.m, w.omegas, w.sources, w.receivers, dirs, alpha=0.5, mu=0.1)
    G = oracle.regulariser(g, 0.5, 0.1)
    for a, t in enumerate(dirs):
        ref = H @ t
        assert np.linalg.norm(hv[a] - ref) / np.linalg.norm(ref) < 1e-6
        np.testing.assert_allclose(hv_reg[a], hv[a] + G @ t, rtol=1e-12)


def test_gn_hessian_symmetric_psd(oracle_mod):
    w = I.small_layered(13, 2, 3, 5, ppws=(9.0,))
    g = Grid.of(w)
    rng = np.random.default_rng(9)
    d1, d2 = rng.standard_normal(g.N), rng.standard_normal(g.N)
    (h1, h2), _ = oracle.gn_hvp(g, w.m, w.omegas, w.sources, w.receivers, [d1, d2])
    assert abs(d2 @ h1 - d1 @ h2) < 1e-10 * abs(d2 @ h1)
    assert d1 @ h1 > 0 and d2 @ h2 > 0


# -------------------------------------------------------------- regulariser --

def test_regulariser_closed_forms(oracle_mod):
    """R = Dx^T Dx + Dz^T Dz with D_n = (n-1) bidiag(1, -1) (eq (ThisGamma)):
    m^T R m for m = a*i + c*j is (n1-1)^2 a^2 (n1-1) n2 + (n2-1)^2 c^2 n1 (n2-1);
    constants are in the kernel; Gamma(0, mu) = mu I."""
    n1, n2 = 6, 4
    g = Grid(n1, n2, 0.2, 0.3)
    R = oracle.regulariser(g, 1.0, 0.0)
    a, c = 0.7, -1.3
    i = np.arange(g.N) % n1
    j = np.arange(g.N) // n1
    mlin = a * i + c * j
    expect = (n1 - 1) ** 2 * a ** 2 * (n1 - 1) * n2 + (n2 - 1) ** 2 * c ** 2 * n1 * (n2 - 1)
    assert mlin @ (R @ mlin) == pytest.approx(expect, rel=1e-13)
    assert np.abs(R @ np.ones(g.N)).max() < 1e-12
    np.testing.assert_allclose(oracle.regulariser(g, 0.0, 0.25).toarray(), 0.25 * np.eye(g.N))


# ------------------------------------------------------------- input checks --

def test_rejects_nonpositive_model(oracle_mod):
    g = Grid(4, 4, 0.1, 0.1)
    m = np.ones(16)
    m[5] = 0.0
    with pytest.raises(ValueError):
        oracle.Factor(g, m, 1.0)
    m[5] = np.nan
    with pytest.raises(ValueError):
        oracle.Factor(g, m, 1.0)
