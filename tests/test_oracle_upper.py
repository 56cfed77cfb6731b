"""Pins of the oracle's sliding-cubic restriction and of the upper-level
derivatives dpsi/dp and dpsi/dalpha.

* the sliding cubic reproduces bicubic polynomials exactly, values and
  derivatives, also where the stencil is moved inward at the edges, and is
  plain sampling at nodes;
* the misfit gradient with off-node sensors against central differences;
* dpsi/dp_{j,l} and dpsi/dalpha against central differences of
  psi = 1/2 ||m' - m_FWI||^2, with m_FWI solved to machine precision by
  Newton's method with the dense Hessian at every perturbed design.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, Sensors
from paper_2301_10762_amd import inputs as I


def test_sliding_cubic_reproduces_bicubics():
    g = Grid(9, 7, 0.3, 0.2)
    rng = np.random.default_rng(0)
    pts = np.column_stack([rng.uniform(0, 8 * 0.3, 40), rng.uniform(0, 6 * 0.2, 40)])
    pts[:4] = [[0.01, 0.02], [2.39, 1.19], [0.05, 1.1], [2.35, 0.1]]   # edge intervals
    S = Sensors(g, pts)
    R0, Rx, Rz = S.matrix(0), S.matrix(1), S.matrix(2)
    x = (np.arange(g.N) % g.nx) * g.hx
    z = (np.arange(g.N) // g.nx) * g.hz
    for a in range(4):
        for b in range(4):
            f = x ** a * z ** b
            px, pz = pts[:, 0], pts[:, 1]
            assert np.allclose(R0 @ f, px ** a * pz ** b, rtol=1e-11, atol=1e-11)
            dfx = a * px ** max(a - 1, 0) * pz ** b if a else 0 * px
            dfz = b * px ** a * pz ** max(b - 1, 0) if b else 0 * pz
            assert np.allclose(Rx @ f, dfx, rtol=1e-10, atol=1e-10)
            assert np.allclose(Rz @ f, dfz, rtol=1e-10, atol=1e-10)


def test_sliding_cubic_at_nodes_is_sampling():
    g = Grid(8, 6, 0.1, 0.25)
    nodes = [0, 7, 9, 20, 47, 33]
    pts = [[(k % g.nx) * g.hx, (k // g.nx) * g.hz] for k in nodes]
    R = Sensors(g, pts).matrix().toarray()
    E = np.zeros_like(R)
    E[np.arange(len(nodes)), nodes] = 1.0
    assert np.max(np.abs(R - E)) < 1e-14


def test_misfit_gradient_with_sensors_central_differences():
    w = I.small_layered(11, 5, 2, 3, ppws=(8.0,))
    g = Grid.of(w)
    h = g.hx
    S = Sensors(g, [[2.3 * h, 0.4 * h], [5.5 * h, 1.7 * h], [8.1 * h, 6.2 * h]])
    d = oracle.synth_data(g, w.m_true, w.omegas, w.sources, S)
    _, grad = oracle.misfit_grad(g, w.m, w.omegas, d, w.sources, S, 1e-3, 1e-4)
    rng = np.random.default_rng(4)
    for _ in range(2):
        dlt = rng.standard_normal(g.N)
        t = 1e-6
        fp, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d, w.sources, S, 1e-3, 1e-4)
        fm, _ = oracle.misfit_grad(g, w.m - t * dlt, w.omegas, d, w.sources, S, 1e-3, 1e-4)
        fd = (fp - fm) / (2 * t)
        assert abs(fd - grad @ dlt) <= 1e-7 * abs(fd)


class _Bilevel:
    """A 9 x 9 training problem: two sources, three off-node sensors, two
    frequencies; m_FWI by Newton's method with the dense full Hessian."""

    def __init__(self):
        w = I.small_layered(9, 3, 2, 3, ppws=(6.0, 9.0))
        self.w, self.g = w, Grid.of(w)
        self.m_train = w.m_true.copy()
        self.src = [int(s) for s in w.sources]
        h = self.g.hx
        self.P = np.array([[2.3 * h, 0.6 * h], [4.7 * h, 1.4 * h], [6.2 * h, 3.3 * h]])
        self.alpha, self.mu = 1e-4, 1e-4

    def hessian(self, m, d, S, alpha):
        return oracle.hvp(self.g, m, self.w.omegas, d, self.src, S, list(np.eye(self.g.N)), alpha, self.mu)

    def fwi(self, P, alpha, m0):
        S = Sensors(self.g, P)
        d = oracle.synth_data(self.g, self.m_train, self.w.omegas, self.src, S)
        m = m0.copy()
        for _ in range(30):
            _, gr = oracle.misfit_grad(self.g, m, self.w.omegas, d, self.src, S, alpha, self.mu)
            if np.linalg.norm(gr) < 1e-13:
                return m, d, S
            m = m - np.linalg.solve(self.hessian(m, d, S, alpha), gr)
        raise AssertionError("Newton did not converge")

    def psi(self, P, alpha, m0):
        return 0.5 * float(np.sum((self.m_train - self.fwi(P, alpha, m0)[0]) ** 2))


@pytest.fixture(scope="module")
def bilevel():
    b = _Bilevel()
    b.m_fwi, d, S = b.fwi(b.P, b.alpha, b.m_train)
    H = b.hessian(b.m_fwi, d, S, b.alpha)
    b.rho = np.linalg.solve(H, b.m_train - b.m_fwi)
    b.S = S
    return b


def upper_fd_errors(b, upper=None):
    upper = upper or oracle.upper_grad
    dp, da = upper(b.g, b.m_fwi, b.m_train, b.w.omegas, b.src, b.S, b.rho)
    t = 1e-5 * b.g.hx
    fd = np.zeros_like(dp)
    for j in range(len(b.P)):
        for col in range(2):
            Pp, Pm = b.P.copy(), b.P.copy()
            Pp[j, col] += t
            Pm[j, col] -= t
            fd[j, col] = (b.psi(Pp, b.alpha, b.m_fwi) - b.psi(Pm, b.alpha, b.m_fwi)) / (2 * t)
    ta = 1e-4 * b.alpha
    fda = (b.psi(b.P, b.alpha + ta, b.m_fwi) - b.psi(b.P, b.alpha - ta, b.m_fwi)) / (2 * ta)
    return np.linalg.norm(fd - dp) / np.linalg.norm(fd), abs(fda - da) / abs(fda)


def test_upper_grad_matches_differences_of_psi(bilevel):
    ep, ea = upper_fd_errors(bilevel)
    assert ep < 1e-7, ep
    assert ea < 1e-7, ea
