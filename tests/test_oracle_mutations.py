"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each test swaps one piece of the oracle for a plausible wrong version (a
dropped term, a wrong sign, a missing conjugate, a transposed operand, an
off-by-one index) and checks that the finite-difference or identity pin that
guards that piece then fails.  The real oracle passes the same checks in
test_oracle.py.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid
from paper_2301_10762_amd import inputs as I


def _fd_gradient_error(seed=4):
    w = I.small_layered(13, seed, 3, 5, ppws=(8.0,))
    g = Grid.of(w)
    d_obs = oracle.synth_data(g, w.m_true, w.omegas, w.sources, w.receivers)
    _, grad = oracle.misfit_grad(g, w.m, w.omegas, d_obs, w.sources, w.receivers)
    rng = np.random.default_rng(1)
    t = 1e-6
    worst = 0.0
    d, b = oracle.weights(g)
    for kind in range(3):
        dlt = rng.standard_normal(g.N) if kind < 2 else np.where(b > 0, 1.0, 0.0)
        dlt /= np.linalg.norm(dlt)
        fp, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d_obs, w.sources, w.receivers)
        fm, _ = oracle.misfit_grad(g, w.m - t * dlt, w.omegas, d_obs, w.sources, w.receivers)
        fd = (fp - fm) / (2 * t)
        worst = max(worst, abs(fd - grad @ dlt) / abs(fd))
    return worst


def test_unmutated_oracle_passes():
    assert _fd_gradient_error() < 1e-6


def test_dropped_boundary_term_caught(monkeypatch):
    d_b = oracle.weights

    def no_boundary(g, m, omega):
        d, _ = d_b(g)
        return omega ** 2 * d + 0j
    monkeypatch.setattr(oracle, "grad_weight", no_boundary)
    assert _fd_gradient_error() > 1e-4


def test_wrong_boundary_sign_caught(monkeypatch):
    def flipped(g, m, omega):
        d, b = oracle.weights(g)
        return omega ** 2 * d - 1j * omega * b / (2.0 * np.sqrt(m))
    monkeypatch.setattr(oracle, "grad_weight", flipped)
    assert _fd_gradient_error() > 1e-4


def test_transpose_instead_of_adjoint_caught(monkeypatch):
    # A^{-T} = A^{-1} for complex-symmetric A: solving with A instead of A^*
    monkeypatch.setattr(oracle.Factor, "adjoint_solve", lambda self, R: self.solve(R))
    assert _fd_gradient_error() > 1e-4


def test_off_by_one_receiver_scatter_caught(monkeypatch):
    real = oracle.restrict_adjoint

    def shifted(Z, receivers, N):
        return real(Z, np.asarray(receivers) + 1, N)
    monkeypatch.setattr(oracle, "restrict_adjoint", shifted)
    assert _fd_gradient_error() > 1e-4


def test_residual_sign_caught(monkeypatch):
    real = oracle.restrict

    def neg(U, receivers):
        return -real(U, receivers)
    # eps = d + R u instead of d - R u changes phi and its gradient inconsistently
    monkeypatch.setattr(oracle, "restrict", neg)
    assert _fd_gradient_error() > 1e-4


def test_gn_missing_conjugate_caught(monkeypatch):
    """H^(1) symmetry fails if z is not conjugated in the final inner product."""
    w = I.small_layered(9, 2, 2, 4, ppws=(9.0,))
    g = Grid.of(w)
    rng = np.random.default_rng(9)
    d1, d2 = rng.standard_normal(g.N), rng.standard_normal(g.N)
    monkeypatch.setattr(np, "conj", lambda x: x)
    (h1, h2), _ = oracle.gn_hvp(g, w.m, w.omegas, w.sources, w.receivers, [d1, d2])
    assert abs(d2 @ h1 - d1 @ h2) > 1e-6 * abs(d2 @ h1)


# ---------------------------------------------------- full Hessian product --

def _mutant_hvp(old, new):
    """oracle.hvp with one source fragment replaced (the planted mistake)."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.hvp))
    assert src.count(old) == 1, old
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["hvp"]


HVP_MUTATIONS = {
    "dropped_h_term": ("out[a] -= np.real(np.sum(hk * mt[None, :] * U * np.conj(Lam), axis=0))", "pass"),
    "h_exponent": ("m ** 1.5", "m ** 0.5"),
    "h_sign": ("hk = (-1j", "hk = (1j"),
    "dropped_v_term": ("out[a] -= np.real(np.sum(gk * V * np.conj(Lam), axis=0))", "pass"),
    "z_rhs_sign": ("- np.conj(gk) * mt[None, :] * Lam", "+ np.conj(gk) * mt[None, :] * Lam"),
    "z_rhs_unconjugated": ("- np.conj(gk) * mt[None, :] * Lam", "- gk * mt[None, :] * Lam"),
    "z_rhs_dropped": ("- np.conj(gk) * mt[None, :] * Lam", ""),
    "forward_instead_of_adjoint": ("Z = F.adjoint_solve(rhs)", "Z = F.solve(rhs)"),
}


@pytest.mark.parametrize("name", sorted(HVP_MUTATIONS))
def test_hvp_mutation_caught(name):
    from tests.test_oracle_hessian import hvp_fd_error
    old, new = HVP_MUTATIONS[name]
    assert hvp_fd_error(_mutant_hvp(old, new)) > 1e-4


# ------------------------------------------------- upper-level derivatives --

def _mutant_upper(old, new):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.upper_grad))
    assert src.count(old) == 1, old
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["upper_grad"]


UPPER_MUTATIONS = {
    # the form printed in eq (gradALT1), without the conjugates of the derivation
    "no_conjugates": ("dtau * np.conj(du) + tau * np.conj(ddu)", "dtau * du + tau * ddu"),
    "dropped_dtau_term": ("dtau * np.conj(du) + tau * np.conj(ddu)", "tau * np.conj(ddu)"),
    "dropped_tau_term": ("dtau * np.conj(du) + tau * np.conj(ddu)", "dtau * np.conj(du)"),
    "tau_without_rho": ("grad_weight(g, m_fwi, w)[None, :] * rho[None, :] * U", "grad_weight(g, m_fwi, w)[None, :] * U"),
    "adjoint_tau": ("Tau = F.solve(", "Tau = F.adjoint_solve("),
    "alpha_with_gamma": ("Rg = regulariser(g, 1.0, 0.0)", "Rg = regulariser(g, 1.0, 1.0)"),
}


@pytest.mark.parametrize("name", sorted(UPPER_MUTATIONS))
def test_upper_mutation_caught(name):
    from tests.test_oracle_upper import _Bilevel, upper_fd_errors
    import numpy as np
    b = _Bilevel()
    b.m_fwi, d, S = b.fwi(b.P, b.alpha, b.m_train)
    b.rho = np.linalg.solve(b.hessian(b.m_fwi, d, S, b.alpha), b.m_train - b.m_fwi)
    b.S = S
    old, new = UPPER_MUTATIONS[name]
    ep, ea = upper_fd_errors(b, _mutant_upper(old, new))
    assert max(ep, ea) > 1e-4, (ep, ea)


# ------------------------------------------------------------------ L-BFGS --

def _mutant_lbfgs(old, new):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.lbfgs))
    assert src.count(old) == 1, old
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["lbfgs"]


LBFGS_MUTATIONS = {
    "first_loop_oldest_first": ("for s, y in zip(reversed(S), reversed(Y)):", "for s, y in zip(S, Y):"),
    "second_loop_sign": ("q += (a_ - b_) * s", "q += (b_ - a_) * s"),
    "memory_never_kept": ("S.append(s_)\n            Y.append(y_)", "pass"),
}


@pytest.mark.parametrize("name", sorted(LBFGS_MUTATIONS))
def test_lbfgs_mutation_caught(name):
    """Each planted mistake breaks the quadratic-termination pin (or stops
    the run short of the solution)."""
    import numpy as np
    old, new = LBFGS_MUTATIONS[name]
    opt = _mutant_lbfgs(old, new)
    rng = np.random.default_rng(12)
    n = 12
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    b = rng.standard_normal(n)
    x, info = opt(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.ones(n), memory=n, max_iters=100, gtol=1e-8,
                  c2=1e-2)
    assert info["status"] != "converged" or info["iterations"] > n + 1


# ------------------------------------------------------------ point sources --

def test_point_source_swapped_local_coordinates_caught():
    """Swapping x and z inside one cut breaks second-order convergence of the
    sensor data."""
    import inspect
    import textwrap
    from tests.test_oracle_offgrid import data_convergence_ratios
    src = textwrap.dedent(inspect.getsource(oracle.point_sources))
    old = "a = {k00: 1 - xi, k10: xi - eta, k11: eta}"
    assert src.count(old) == 1
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, "a = {k00: 1 - eta, k10: eta - xi, k11: xi}"), "<mutant>", "exec"), ns)
    r1, r2 = data_convergence_ratios(ns["point_sources"])
    assert not (3.5 <= r1 <= 6.0 and 3.5 <= r2 <= 6.0), (r1, r2)
