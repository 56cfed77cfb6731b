"""Pins of the oracle's point sources between nodes, of data at points on
grids that differ from the inversion grid, and of h_x != h_z.

* the hat-function load is a partition of unity, reproduces linear
  functions exactly, is e_s at a node and is symmetric under reflection;
* sensor data from a source and sensors between nodes converge at second
  order under refinement: errors against the finest grid shrink by about 4
  per halving of h (first order would give about 2);
* the misfit gradient with h_x != h_z, point sources and sensors at points
  against central differences.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid


def _pts(g, n, seed):
    rng = np.random.default_rng(seed)
    return np.column_stack([rng.uniform(0, (g.nx - 1) * g.hx, n), rng.uniform(0, (g.nz - 1) * g.hz, n)])


def test_point_sources_partition_of_unity_and_linear_reproduction():
    g = Grid(9, 7, 0.3, 0.2)
    P = _pts(g, 50, 0)
    P[:3] = [[0.0, 0.0], [2.4, 1.2], [2.4, 0.0]]
    E = oracle.point_sources(g, P).real
    x = (np.arange(g.N) % g.nx) * g.hx
    z = (np.arange(g.N) // g.nx) * g.hz
    assert np.allclose(E.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(E @ x, P[:, 0], atol=1e-13)
    assert np.allclose(E @ z, P[:, 1], atol=1e-13)
    assert np.all(E >= -1e-15)


def test_point_sources_at_nodes_and_reflection():
    g = Grid(8, 6, 0.1, 0.25)
    nodes = [0, 7, 9, 20, 47, 33]
    pts = [[(k % g.nx) * g.hx, (k // g.nx) * g.hz] for k in nodes]
    assert np.array_equal(oracle.point_sources(g, pts), oracle.unit_sources(g, nodes))
    P = _pts(g, 20, 3)
    E = oracle.point_sources(g, P).real.reshape(-1, g.nz, g.nx)
    Pm = P.copy()
    Pm[:, 0] = (g.nx - 1) * g.hx - P[:, 0]
    Em = oracle.point_sources(g, Pm).real.reshape(-1, g.nz, g.nx)
    assert np.allclose(E, Em[:, :, ::-1], atol=1e-14)


def data_convergence_ratios(point_sources=None):
    """Errors of the sensor data on n = 21, 41, 81 against n = 161 (one point
    source, three sensors, all between nodes, constant c = 2, 4 Hz)."""
    L, c, omega = 0.5, 2.0, 2 * np.pi * 4
    ds = []
    for n in (21, 41, 81, 161):
        h = L / (n - 1)
        g = Grid(n, n, h, h)
        m = np.full(g.N, 1 / c ** 2)
        S = oracle.Sensors(g, [[0.3711, 0.2513], [0.1033, 0.4122], [0.4411, 0.0617]])
        E = (point_sources or oracle.point_sources)(g, [[0.2137, 0.1311]])
        F = oracle.Factor(g, m, omega)
        ds.append(oracle.restrict(F.solve(E), S)[0])
        F.close()
    e = [np.linalg.norm(ds[i] - ds[-1]) for i in range(3)]
    return e[0] / e[1], e[1] / e[2]


def test_data_between_nodes_converge_at_second_order():
    r1, r2 = data_convergence_ratios()
    assert 3.5 <= r1 <= 6.0 and 3.5 <= r2 <= 6.0, (r1, r2)


def test_gradient_with_unequal_spacing_and_points():
    from paper_2301_10762_amd import inputs as I
    w = I.small_layered(12, 8, 2, 3, ppws=(8.0,))
    g = Grid(w.nx, w.nz, w.hx, 0.6 * w.hz)
    src = _pts(g, 2, 5) * [1.0, 0.3]
    S = oracle.Sensors(g, _pts(g, 4, 6) * [1.0, 0.5] + [0.0, 0.4 * (g.nz - 1) * g.hz])
    d = oracle.synth_data(g, w.m_true, w.omegas, src, S)
    _, grad = oracle.misfit_grad(g, w.m, w.omegas, d, src, S, 1e-3, 1e-4)
    rng = np.random.default_rng(2)
    for _ in range(2):
        dlt = rng.standard_normal(g.N)
        t = 1e-6
        fp, _ = oracle.misfit_grad(g, w.m + t * dlt, w.omegas, d, src, S, 1e-3, 1e-4)
        fm, _ = oracle.misfit_grad(g, w.m - t * dlt, w.omegas, d, src, S, 1e-3, 1e-4)
        assert abs((fp - fm) / (2 * t) - grad @ dlt) <= 1e-7 * abs((fp - fm) / (2 * t))
