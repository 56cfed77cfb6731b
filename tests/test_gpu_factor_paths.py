"""GPU: the two factorisation schedules give the same factors.

The persistent schedule (one launch per group, every workgroup resident,
panel data exchanged through memory between the workgroups of a front) and
the launch-per-panel-step schedule perform the same arithmetic in the same
order on every element, so their solutions must agree bitwise; both are also
checked against the FP64 oracle, including ragged grids, both fronts of the
twisted factorisation, the merge row, complex64 factors with refinement and
forced tile pivoting.
"""
import numpy as np
import pytest

import oracle
from paper_2301_10762_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    yield h
    h.set_factor_path(False)
    h.set_tile_pivoting(False)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (nx, nz, hx, hz): several tiles with tails, short and tall grids, the
# smallest grids with and without a bottom front
GRIDS = [(40, 23, 0.05, 0.04), (17, 13, 0.06, 0.06), (70, 9, 0.03, 0.05), (130, 33, 0.02, 0.02),
         (16, 5, 0.1, 0.1), (16, 4, 0.1, 0.1), (2, 3, 0.5, 0.5)]


def _system(nx, nz, hx, hz, seed, S=7):
    rng = np.random.default_rng(seed)
    m = 0.2 + 0.05 * rng.random(nx * nz)
    w = 2 * np.pi * 2.5
    B = (rng.standard_normal((S, nx * nz)) + 1j * rng.standard_normal((S, nx * nz)))
    return m, w, B


def _solve(helm, grid, m, w, B, precision, persistent):
    helm.set_factor_path(persistent)
    before = helm.counters()["launches"]
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    launches = helm.counters()["launches"] - before
    X, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    F.close()
    return X.cpu().numpy(), info, launches


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("nx,nz,hx,hz", GRIDS)
def test_paths_agree_and_match_oracle(helm, nx, nz, hx, hz, precision):
    m, w, B = _system(nx, nz, hx, hz, seed=nx * 100 + nz)
    grid = helm.Grid(nx, nz, hx, hz)
    print(f"grid {nx}x{nz} {precision}", flush=True)
    Xp, ip, lp = _solve(helm, grid, m, w, B, precision, True)
    Xs, is_, ls = _solve(helm, grid, m, w, B, precision, False)
    assert lp < ls                      # the persistent schedule was used
    assert helm.counters()["persist_fallbacks"] == 0
    if precision == "fp64":
        assert np.array_equal(Xp, Xs)
    g = oracle.Grid(nx, nz, hx, hz)
    Fo = oracle.Factor(g, m, w)
    Xo = Fo.solve(B)
    Fo.close()
    assert rel(Xp, Xo) < 1e-9 and rel(Xs, Xo) < 1e-9
    assert ip.max_relres <= 1e-10 and is_.max_relres <= 1e-10


@pytest.mark.parametrize("persistent,precision", [(True, "fp64"), (False, "fp64"), (False, "fp32_ir")])
def test_batch_of_mixed_grids(helm, persistent, precision):
    """Fronts of different widths in one launch: the persistent schedule, and
    the step launches with their scanned front lookup."""
    helm.set_factor_path(persistent)
    before = helm.counters()["persist_fallbacks"]
    specs = [GRIDS[0], GRIDS[1], GRIDS[3], GRIDS[5]]
    grids, ms, ws, Bs = [], [], [], []
    for k, (nx, nz, hx, hz) in enumerate(specs):
        m, w, B = _system(nx, nz, hx, hz, seed=7 + k, S=3 + k)
        grids.append(helm.Grid(nx, nz, hx, hz))
        ms.append(torch.as_tensor(m, device="cuda"))
        ws.append(w * (1 + 0.1 * k))
        Bs.append(torch.as_tensor(B, device="cuda"))
    Fs = helm.factor_batch(grids, ms, ws, precision)
    Xs, infos = helm.solve_batch(Fs, Bs, tol=1e-10)
    for F, X, B, m, w, g, info in zip(Fs, Xs, Bs, ms, ws, grids, infos):
        og = oracle.Grid(g.nx, g.nz, g.hx, g.hz)
        Fo = oracle.Factor(og, m.cpu().numpy(), w)
        assert rel(X.cpu().numpy(), Fo.solve(B.cpu().numpy())) < 1e-9
        Fo.close()
        F.close()
        assert info.max_relres <= 1e-10
    assert helm.counters()["persist_fallbacks"] == before
    helm.set_factor_path(False)


def test_persistent_with_forced_tile_pivoting(helm):
    nx, nz, hx, hz = GRIDS[0]
    m, w, B = _system(nx, nz, hx, hz, seed=3)
    grid = helm.Grid(nx, nz, hx, hz)
    helm.set_tile_pivoting(True)
    try:
        Xp, ip, _ = _solve(helm, grid, m, w, B, "fp64", True)
        Xs, _, _ = _solve(helm, grid, m, w, B, "fp64", False)
    finally:
        helm.set_tile_pivoting(False)
        helm.set_factor_path(False)
    assert np.array_equal(Xp, Xs)
    g = oracle.Grid(nx, nz, hx, hz)
    Fo = oracle.Factor(g, m, w)
    assert rel(Xp, Fo.solve(B)) < 1e-9
    Fo.close()


def test_block_cache_reuses_freed_factor_memory(helm):
    """A destroyed factor's memory goes to the library's block cache and the
    next factorisation of the same size takes it: the cache shrinks, and the
    result is bitwise the one computed on fresh memory.  A zero limit empties
    the cache."""
    nx, nz, hx, hz = 130, 33, 0.02, 0.02
    m, w, B = _system(nx, nz, hx, hz, seed=11)
    grid = helm.Grid(nx, nz, hx, hz)
    Bd = torch.as_tensor(B, device="cuda")
    md = torch.as_tensor(m, device="cuda")
    old = helm.set_cache_limit(0)
    try:
        helm.set_cache_limit(1 << 34)
        F = helm.factor(grid, md, w, "fp32_ir")
        X1, _ = helm.solve(F, Bd, tol=1e-10)
        X1 = X1.cpu().numpy()
        F.close()
        torch.cuda.synchronize()
        held = helm.counters()["cached_bytes"]
        assert held >= 144 * 144 * 33 * 8   # at least this factor's G (np = 144) went to the cache
        F = helm.factor(grid, md, w, "fp32_ir")
        assert helm.counters()["cached_bytes"] < held
        X2, info = helm.solve(F, Bd, tol=1e-10)
        F.close()
        assert np.array_equal(X2.cpu().numpy(), X1)
        assert info.max_relres <= 1e-10
        helm.set_cache_limit(0)
        assert helm.counters()["cached_bytes"] == 0
    finally:
        helm.set_cache_limit(old)
