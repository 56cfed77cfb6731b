"""Pins of the oracle's frequency continuation and of its relative residual.

Frequency continuation (App. "Bilevel Frequency Continuation", Algorithm 2,
its lower level): FWI runs over groups of frequencies in turn, each group from
the model the previous group ended at.  The pin does not rerun that loop.  It
checks the run against quantities computed another way:

* each group ends at the minimiser of its own objective (its frequencies and
  their data only), found by Newton's method with the dense full Hessian;
* each group starts where the previous group's minimiser is: its first
  objective value equals that objective evaluated directly at the previous
  minimiser (the first group's equals it at m0).

Two plausible mistakes in the loop must fail the pin: restarting every group
from m0, and taking a group's data by its position in the list of groups
instead of by frequency index.

Relative residual (the IR acceptance test, max_s ||b_s - A x_s|| / ||b_s||):
pinned against the operator assembled element by element (tests/fem_p1.py),
with the forward and the adjoint operator.  A wrong denominator (the norm of
all columns together, or ||x||) and the transpose in place of the adjoint
must fail the pin.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, Sensors
from paper_2301_10762_amd import inputs as I
from tests import fem_p1

# ------------------------------------------------------------ continuation --


class _Problem:
    """9 x 9 grid, two frequencies (PPW 6 and 9), two sources, three sensors
    between nodes, data from the true model; alpha = mu = 1e-4."""

    def __init__(self):
        w = I.small_layered(9, 3, 2, 3, ppws=(6.0, 9.0))
        self.w, self.g = w, Grid.of(w)
        self.src = [int(s) for s in w.sources]
        h = self.g.hx
        self.S = Sensors(self.g, [[2.3 * h, 0.6 * h], [4.7 * h, 1.4 * h], [6.2 * h, 3.3 * h]])
        self.alpha, self.mu = 1e-4, 1e-4
        self.omegas = list(w.omegas)
        self.d = oracle.synth_data(self.g, w.m_true, self.omegas, self.src, self.S)
        self.m0 = w.m_true + 0.05 * (w.m - w.m_true)

    def objective(self, m, freqs):
        """phi over the frequencies `freqs` (indices) with their own data."""
        return oracle.misfit_grad(self.g, m, [self.omegas[i] for i in freqs], self.d[list(freqs)], self.src,
                                  self.S, self.alpha, self.mu)

    def newton(self, freqs, m0):
        """Minimiser of objective(., freqs) by Newton's method, dense Hessian."""
        om = [self.omegas[i] for i in freqs]
        d = self.d[list(freqs)]
        m = np.array(m0, dtype=np.float64)
        for _ in range(40):
            _, gr = self.objective(m, freqs)
            if np.linalg.norm(gr) < 1e-13:
                return m
            H = oracle.hvp(self.g, m, om, d, self.src, self.S, list(np.eye(self.g.N)), self.alpha, self.mu)
            m = m - np.linalg.solve(H, gr)
        raise AssertionError("Newton did not converge")


GROUPS = [[1], [0, 1]]   # lower frequency (PPW 9) first, then both


@pytest.fixture(scope="module")
def prob():
    p = _Problem()
    p.minimisers = []
    start = p.m0
    for grp in GROUPS:
        start = p.newton(grp, start)
        p.minimisers.append(start)
    return p


def continuation_errors(p, run=None):
    """Deviations of a continuation run from the independently computed
    minimisers and starting values; every entry must be small."""
    run = run or oracle.fwi_continuation
    m, infos = run(p.g, p.m0, GROUPS, p.omegas, p.d, p.src, p.S, p.alpha, p.mu, memory=8, max_iters=400,
                   gtol=1e-7)
    err = {}
    starts = [p.m0] + p.minimisers[:-1]
    for k, (grp, info) in enumerate(zip(GROUPS, infos)):
        f_start, _ = p.objective(starts[k], grp)
        f_min, _ = p.objective(p.minimisers[k], grp)
        err[f"start{k}"] = abs(info["f0"] - f_start) / abs(f_start)
        err[f"end{k}"] = abs(info["f"] - f_min) / abs(f_min)
    err["model"] = float(np.linalg.norm(m - p.minimisers[-1]) / np.linalg.norm(p.minimisers[-1]))
    return err


def test_minimisers_differ_between_groups(prob):
    # the pin can only see a wrong start or wrong data if the groups' objectives differ
    a, b = prob.minimisers
    assert np.linalg.norm(a - b) > 1e-3 * np.linalg.norm(b)
    f_m0, _ = prob.objective(prob.m0, GROUPS[1])
    f_a, _ = prob.objective(a, GROUPS[1])
    assert abs(f_m0 - f_a) > 0.5 * abs(f_a)


def test_continuation_matches_group_minimisers(prob):
    err = continuation_errors(prob)
    assert err["model"] <= 1e-6, err
    for k in range(len(GROUPS)):
        # a group's start model is the previous group's L-BFGS result, which
        # is within 1e-6 of the Newton minimiser; phi there differs by O(|grad| 1e-6)
        assert err[f"start{k}"] <= 1e-4, err
        assert err[f"end{k}"] <= 1e-8, err


def _restart_from_m0(g, m0, groups, omegas, d_obs, sources, receivers, alpha=0.0, mu=0.0, **opts):
    m, infos = None, []
    for grp in groups:
        idx = [int(i) for i in grp]
        m, info = oracle.fwi(g, np.array(m0, dtype=np.float64), [omegas[i] for i in idx], np.asarray(d_obs)[idx],
                             sources, receivers, alpha, mu, **opts)
        infos.append(info)
    return m, infos


def _data_by_position(g, m0, groups, omegas, d_obs, sources, receivers, alpha=0.0, mu=0.0, **opts):
    m, infos = np.array(m0, dtype=np.float64), []
    for grp in groups:
        idx = [int(i) for i in grp]
        m, info = oracle.fwi(g, m, [omegas[i] for i in idx], np.asarray(d_obs)[:len(idx)], sources, receivers,
                             alpha, mu, **opts)
        infos.append(info)
    return m, infos


@pytest.mark.parametrize("mutant", [_restart_from_m0, _data_by_position], ids=["restart_from_m0", "data_by_position"])
def test_continuation_mutation_caught(prob, mutant):
    err = continuation_errors(prob, mutant)
    worst = max(err[f"start{k}"] for k in range(len(GROUPS)))
    worst = max(worst, max(err[f"end{k}"] for k in range(len(GROUPS))) * 1e4)
    assert worst > 1e-2, err


# ---------------------------------------------------------------- relres --


def _relres_reference(w, X, B, adjoint):
    """max-free per-column ||B - A X|| / ||B|| with A from element assembly."""
    A, *_ = fem_p1.operator(w.nx, w.nz, w.hx, w.hz, w.m, w.omegas[0])
    A = A.toarray()
    Aop = A.conj().T if adjoint else A
    R = B - X @ Aop.T
    return np.linalg.norm(R, axis=1) / np.linalg.norm(B, axis=1)


def relres_errors(relres=None):
    relres = relres or oracle.relres
    w = I.small_layered(10, 7, 2, 3, ppws=(7.0,))
    g = Grid.of(w)
    rng = np.random.default_rng(11)
    S = 5
    # columns of very different size and residual, so that per-column
    # normalisation matters
    scale = 10.0 ** np.arange(-2, 3)
    B = (rng.standard_normal((S, g.N)) + 1j * rng.standard_normal((S, g.N))) * scale[:, None]
    out = 0.0
    for adjoint in (False, True):
        F = oracle.Factor(g, w.m, w.omegas[0])
        X = F.adjoint_solve(B) if adjoint else F.solve(B)
        F.close()
        X = X + 1e-3 * rng.standard_normal(X.shape) * np.abs(X).max(axis=1, keepdims=True)
        ref = _relres_reference(w, X, B, adjoint)
        got = relres(g, w.m, w.omegas[0], X, B, adjoint=adjoint)
        out = max(out, float(np.max(np.abs(got - ref) / ref)))
    return out


def test_relres_matches_assembled_operator():
    assert relres_errors() <= 1e-10


def _frobenius_denominator(g, m, omega, X, B, adjoint=False):
    B = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    R = B - oracle.apply(g, m, omega, X, adjoint)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(B)


def _solution_denominator(g, m, omega, X, B, adjoint=False):
    B = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    R = B - oracle.apply(g, m, omega, X, adjoint)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(np.atleast_2d(X), axis=1)


def _transpose_for_adjoint(g, m, omega, X, B, adjoint=False):
    B = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    R = B - oracle.apply(g, m, omega, X, False)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(B, axis=1)


@pytest.mark.parametrize("mutant", [_frobenius_denominator, _solution_denominator, _transpose_for_adjoint],
                         ids=["frobenius_denominator", "solution_denominator", "transpose_for_adjoint"])
def test_relres_mutation_caught(mutant):
    assert relres_errors(mutant) > 1e-2
