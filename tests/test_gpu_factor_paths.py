"""GPU: the launch-per-panel-step factorisation on awkward shapes.

Grids with ragged tiles, short and tall grids, the smallest grids with and
without a bottom front (the two-ended elimination and its merge row), fronts
of different widths in one launch (the scanned front lookup), complex64
factors with refinement and forced tile pivoting: every solution column is
compared with the FP64 oracle, and the number of launches is the schedule's
(one initial launch, then one per panel step of the longest front).  The
device block cache is checked to give bitwise the result computed on fresh
memory.
"""
import numpy as np
import pytest

import oracle
from tests.parity import assert_cols

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    yield h
    h.set_tile_pivoting(False)


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


def _steps(nx, nz):
    """Panel-step launches of one system: the top front's blocks (rows 0..k,
    k = ceil((nz + 1) / 2) when a bottom front exists) times panels per block."""
    np_ = (nx + 15) // 16 * 16
    npan = (np_ + 31) // 32
    k = (nz + 1) // 2
    if nz - 1 - k < 1:
        k = nz - 1
    return npan * (k + 1)


def _oracle(nx, nz, hx, hz, m, w, B):
    Fo = oracle.Factor(oracle.Grid(nx, nz, hx, hz), m, w)
    Xo = Fo.solve(B)
    Fo.close()
    return Xo


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("nx,nz,hx,hz", GRIDS)
def test_step_schedule_matches_oracle(helm, nx, nz, hx, hz, precision):
    m, w, B = _system(nx, nz, hx, hz, seed=nx * 100 + nz)
    grid = helm.Grid(nx, nz, hx, hz)
    print(f"grid {nx}x{nz} {precision}", flush=True)
    before = helm.counters()["launches"]
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    launches = helm.counters()["launches"] - before
    X, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    F.close()
    # zeroing + model check, then the table upload, the initial launch and the
    # panel steps; a group whose unpivoted tiles met a small pivot is factored
    # again with pivoting inside the tiles
    T = _steps(nx, nz)
    assert launches in (4 + T, 6 + 2 * T), (launches, T)
    assert_cols(X.cpu().numpy(), _oracle(nx, nz, hx, hz, m, w, B), 1e-9, what=f"{nx}x{nz} {precision}")
    assert info.max_relres <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_of_mixed_grids(helm, precision):
    """Fronts of different widths in one launch (the scanned front lookup)."""
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
        Xo = _oracle(g.nx, g.nz, g.hx, g.hz, m.cpu().numpy(), w, B.cpu().numpy())
        assert_cols(X.cpu().numpy(), Xo, 1e-9, what=f"{g.nx}x{g.nz} in a mixed batch")
        F.close()
        assert info.max_relres <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_forced_tile_pivoting(helm, precision):
    nx, nz, hx, hz = GRIDS[0]
    m, w, B = _system(nx, nz, hx, hz, seed=3)
    grid = helm.Grid(nx, nz, hx, hz)
    helm.set_tile_pivoting(True)
    try:
        F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
        X, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
        F.close()
    finally:
        helm.set_tile_pivoting(False)
    assert_cols(X.cpu().numpy(), _oracle(nx, nz, hx, hz, m, w, B), 1e-9, what="forced pivoting")
    assert info.max_relres <= 1e-10


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
