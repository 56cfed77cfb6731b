"""Pins of the oracle's L-BFGS / strong-Wolfe optimiser and of FWI built on it.

* Rosenbrock's function from (-1.2, 1): the minimiser (1, 1);
* SPD quadratics: with memory n and a near-exact line search (c2 = 1e-2)
  the quasi-Newton method converges in at most n + 1 iterations (BFGS with
  exact line searches terminates in n; steepest descent would need hundreds);
  with memory 3 it still converges to the solution of the linear system;
* every accepted step satisfies the strong Wolfe conditions;
* FWI on a 9 x 9 problem with sensors between nodes converges to the
  minimiser found by Newton's method with the dense full Hessian.
"""
import numpy as np
import pytest

import oracle


def _rosen(x):
    f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
    return f, g


def test_rosenbrock():
    x, info = oracle.lbfgs(_rosen, [-1.2, 1.0], max_iters=200, gtol=1e-10)
    assert info["status"] == "converged"
    assert np.max(np.abs(x - 1.0)) < 1e-8


def _quadratic(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    b = rng.standard_normal(n)
    return A, b, np.linalg.solve(A, b)


@pytest.mark.parametrize("n", [6, 12])
def test_quadratic_termination(n):
    A, b, xs = _quadratic(n, n)
    x, info = oracle.lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.ones(n), memory=n, max_iters=100,
                           gtol=1e-8, c2=1e-2)
    assert info["status"] == "converged"
    assert info["iterations"] <= n + 1
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs) * np.linalg.cond(A)


def test_quadratic_limited_memory():
    A, b, xs = _quadratic(30, 1)
    x, info = oracle.lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.ones(30), memory=3, max_iters=300,
                           gtol=1e-9)
    assert info["status"] == "converged"
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_accepted_steps_satisfy_strong_wolfe():
    c1, c2 = 1e-4, 0.9
    seen = {}

    def fg(x):
        f, g = _rosen(x)
        seen[tuple(x)] = (f, g)
        return f, g
    # the accepted iterates are the evaluated points whose f is in the history
    x, info = oracle.lbfgs(fg, np.array([-1.2, 1.0]), max_iters=30, gtol=1e-10, c1=c1, c2=c2)
    by_f = {float(v[0]): np.array(k) for k, v in seen.items()}
    iterates = [by_f[float(h)] for h in info["history"]]
    for xa, xb in zip(iterates[:-1], iterates[1:]):
        fa, ga = _rosen(xa)
        fb, gb = _rosen(xb)
        s = xb - xa
        assert fb <= fa + c1 * (ga @ s) + 1e-15 * abs(fa)
        assert abs(gb @ s) <= c2 * abs(ga @ s) * (1 + 1e-12)


def test_fwi_reaches_newton_minimiser():
    from tests.test_oracle_upper import _Bilevel
    b = _Bilevel()
    m_newton, d, S = b.fwi(b.P, b.alpha, b.m_train)
    start = b.m_train + 0.05 * (b.w.m - b.m_train)
    m, info = oracle.fwi(b.g, start, b.w.omegas, d, b.src, S, b.alpha, b.mu, memory=8, max_iters=400, gtol=1e-7)
    assert info["status"] == "converged", info["status"]
    # ||g|| / lambda_min(H) bounds the distance to the minimiser
    assert np.linalg.norm(m - m_newton) <= 1e-6 * np.linalg.norm(m_newton)
