"""GPU: edge cases of the solve entry points, through the C ABI.

* A leading dimension larger than nx*nz (padded by an odd count): the
  padding of X is left untouched and the solution is bitwise the one with
  ld = nx*nz, forward and adjoint, in both precisions.
* Column counts 1, 17 and 200 (one, two and thirteen 16-column tiles, the
  last one ragged) against the FP64 oracle, column by column.
* The smallest grids (2 x 2, 3 x 2) and a tall grid of single-tile blocks
  (2 x 3000: every block is one 16 x 16 tile holding a 2 x 2 system and an
  identity tail) against the oracle.
* The widest grid the library accepts (nx = 8192, three rows; the oracle's
  banded LU cannot factor it in reasonable time): A x = b holds to the
  requested tolerance by the oracle's own operator, and the complex128 and
  refined complex64 solutions agree.
* Calls with no columns, a negative count, ld below nx*nz or an empty
  batch are rejected with HELM_EINVAL before any launch.
* One batched solve over complex128 and complex64 factors gives each
  factor bitwise its result in a batch of its own precision, forward and
  adjoint.
* A solve on a stream other than the current one sees a right-hand side
  whose writer was still queued on the current stream (behind a bounded
  sleep kernel) when the call was made: the binding orders the side stream
  after the current one.
* Releasing a factor returns without waiting for the GPU, yet its memory
  is not reused before a solve still queued on another stream has read it:
  a new factor made at once on the released factor's stream (which takes
  over that memory) leaves the queued solve's result bitwise unchanged.
"""
import ctypes
import time

import numpy as np
import pytest

import oracle
from tests.parity import assert_cols

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECISIONS = ["fp64", "fp32_ir"]


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    return h


def _system(nx, nz, seed, S):
    rng = np.random.default_rng(seed)
    m = 0.2 + 0.05 * rng.random(nx * nz)
    B = rng.standard_normal((S, nx * nz)) + 1j * rng.standard_normal((S, nx * nz))
    return m, 2 * np.pi * 2.5, B


def _oracle_solve(g, m, w, B, adjoint=False):
    Fo = oracle.Factor(g, m, w)
    X = Fo.adjoint_solve(B) if adjoint else Fo.solve(B)
    Fo.close()
    return X


def _raw_solve(helm, F, B, X, S, ld, adjoint, tol):
    """helm_solve / helm_adjoint_solve on raw device buffers of S columns of ld."""
    info = helm._Info()
    call = helm.lib().helm_adjoint_solve if adjoint else helm.lib().helm_solve
    rc = call(F.handle, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()), S, ld, float(tol),
              helm._stream(None), ctypes.byref(info))
    return rc, helm.Info.of(info)


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_padded_leading_dimension(helm, precision, adjoint):
    nx, nz, S, pad = 37, 29, 5, 7
    N = nx * nz
    ld = N + pad
    m, w, B = _system(nx, nz, 21, S)
    grid = helm.Grid(nx, nz, 0.04, 0.03)
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    print(f"padded ld {ld} (N {N}), {precision}, adjoint {adjoint}", flush=True)
    Bp = torch.full((S, ld), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    Bp[:, :N] = torch.as_tensor(B, device="cuda")
    sentinel = complex(12345.0, -6789.0)
    Xp = torch.full((S, ld), sentinel, dtype=torch.complex128, device="cuda")
    rc, info = _raw_solve(helm, F, Bp, Xp, S, ld, adjoint, 1e-10)
    assert rc == 0, helm.lib().helm_last_error()
    Xref, _ = (helm.adjoint_solve if adjoint else helm.solve)(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    F.close()
    torch.cuda.synchronize()
    assert torch.equal(Xp[:, :N], Xref)                           # bitwise the unpadded solve
    assert bool((Xp[:, N:] == sentinel).all())                    # the padding is not written
    assert info.max_relres <= 1e-10
    Xo = _oracle_solve(oracle.Grid(nx, nz, 0.04, 0.03), m, w, B, adjoint)
    assert_cols(Xp[:, :N].cpu().numpy(), Xo, 1e-9, what=f"ld {ld}")


@pytest.mark.parametrize("S", [1, 17, 200])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_column_counts(helm, precision, S):
    nx, nz = 23, 19
    m, w, B = _system(nx, nz, 100 + S, S)
    grid = helm.Grid(nx, nz, 0.05, 0.05)
    print(f"{S} columns, {precision}", flush=True)
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    X, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    F.close()
    assert X.shape == (S, nx * nz)
    assert info.max_relres <= 1e-10
    assert_cols(X.cpu().numpy(), _oracle_solve(oracle.Grid(nx, nz, 0.05, 0.05), m, w, B), 1e-9, what=f"S={S}")


@pytest.mark.parametrize("nx,nz,h", [(2, 2, 0.5), (3, 2, 0.4), (2, 3000, 0.01)])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_smallest_and_tall_grids(helm, precision, nx, nz, h):
    m, w, B = _system(nx, nz, nx * 7 + nz, 3)
    grid = helm.Grid(nx, nz, h, h)
    print(f"grid {nx}x{nz}, {precision}", flush=True)
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    X, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    L, linfo = helm.adjoint_solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
    F.close()
    assert info.max_relres <= 1e-10 and linfo.max_relres <= 1e-10
    g = oracle.Grid(nx, nz, h, h)
    assert_cols(X.cpu().numpy(), _oracle_solve(g, m, w, B), 1e-9, what=f"{nx}x{nz}")
    assert_cols(L.cpu().numpy(), _oracle_solve(g, m, w, B, adjoint=True), 1e-9, what=f"{nx}x{nz} adjoint")


def test_widest_grid(helm):
    nx, nz, h, S = 8192, 3, 0.025, 4
    m = np.full(nx * nz, 0.25)                  # 2 km/s
    w = 2 * np.pi * 2.0 / (20 * h)              # 20 points per wavelength
    rng = np.random.default_rng(5)
    B = rng.standard_normal((S, nx * nz)) + 1j * rng.standard_normal((S, nx * nz))
    grid = helm.Grid(nx, nz, h, h)
    g = oracle.Grid(nx, nz, h, h)
    X = {}
    for precision in PRECISIONS:
        print(f"grid {nx}x{nz}, {precision}", flush=True)
        F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
        Xd, info = helm.solve(F, torch.as_tensor(B, device="cuda"), tol=1e-10)
        F.close()
        X[precision] = Xd.cpu().numpy()
        assert info.max_relres <= 1e-10
        rr = oracle.relres(g, m, w, X[precision], B)             # the oracle's own operator
        assert rr.max() <= 1e-10, (precision, rr.max())
    assert_cols(X["fp32_ir"], X["fp64"], 1e-8, what="complex64 + refinement against complex128")


def test_rejects_empty_and_bad_counts(helm):
    nx, nz = 9, 7
    N = nx * nz
    grid = helm.Grid(nx, nz, 0.1, 0.1)
    F = helm.factor(grid, torch.full((N,), 0.25, dtype=torch.float64, device="cuda"), 3.0)
    B = torch.zeros(2, N, dtype=torch.complex128, device="cuda")
    X = torch.zeros_like(B)
    for S, ld in [(0, N), (-1, N), (2, N - 1)]:
        rc, _ = _raw_solve(helm, F, B, X, S, ld, False, 0.0)
        assert rc == helm.EINVAL, (S, ld)
        rc, _ = _raw_solve(helm, F, B, X, S, ld, True, 0.0)
        assert rc == helm.EINVAL, (S, ld)
    L = helm.lib()
    n0 = ctypes.c_int32(0)
    fs = (ctypes.c_void_p * 1)(F.handle)
    ps = (ctypes.c_void_p * 1)(B.data_ptr())
    xs = (ctypes.c_void_p * 1)(X.data_ptr())
    ss = (ctypes.c_int32 * 1)(2)
    lds = (ctypes.c_int64 * 1)(N)
    assert L.helm_solve_batch(n0, fs, ps, xs, ss, lds, 0, 0.0, helm._stream(None), None) == helm.EINVAL
    ss[0] = 0
    assert L.helm_solve_batch(ctypes.c_int32(1), fs, ps, xs, ss, lds, 0, 0.0, helm._stream(None), None) == helm.EINVAL
    F.close()
    assert bool((X == 0).all())                                   # nothing was written


@pytest.mark.parametrize("adjoint", [False, True])
def test_solve_batch_mixes_precisions(helm, adjoint):
    """One helm_solve_batch call over complex128 and complex64 factors (the
    library splits it by precision; each group shares its sweep launches):
    every result is bitwise the same as that factor's solve within a batch of
    its own precision, and matches the oracle."""
    specs = [(23, 19, "fp64"), (17, 13, "fp32_ir"), (30, 11, "fp64"), (9, 25, "fp32_ir")]
    Fs, Bs, data = [], [], []
    for k, (nx, nz, prec) in enumerate(specs):
        m, w, B = _system(nx, nz, 300 + k, 2 + k)
        Fs.append(helm.factor(helm.Grid(nx, nz, 0.05, 0.05), torch.as_tensor(m, device="cuda"), w, prec))
        Bs.append(torch.as_tensor(B, device="cuda"))
        data.append((nx, nz, m, w, B))
    print(f"mixed-precision batch, adjoint {adjoint}", flush=True)
    Xm, infos = helm.solve_batch(Fs, Bs, adjoint=adjoint, tol=1e-10)
    for prec in ("fp64", "fp32_ir"):
        idx = [k for k, sp in enumerate(specs) if sp[2] == prec]
        Xs, _ = helm.solve_batch([Fs[k] for k in idx], [Bs[k] for k in idx], adjoint=adjoint, tol=1e-10)
        for k, X in zip(idx, Xs):
            assert torch.equal(Xm[k], X), (k, prec)
    for F, X, info, (nx, nz, m, w, B) in zip(Fs, Xm, infos, data):
        F.close()
        assert info.max_relres <= 1e-10
        Xo = _oracle_solve(oracle.Grid(nx, nz, 0.05, 0.05), m, w, B, adjoint)
        assert_cols(X.cpu().numpy(), Xo, 1e-9, what=f"{nx}x{nz} in a mixed-precision batch")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_side_stream_waits_for_inputs(helm, precision):
    nx, nz, S = 23, 19, 4
    m, w, B = _system(nx, nz, 77, S)
    grid = helm.Grid(nx, nz, 0.05, 0.05)
    F = helm.factor(grid, torch.as_tensor(m, device="cuda"), w, precision)
    B0 = torch.as_tensor(B, device="cuda")
    Xref, _ = helm.solve(F, B0, tol=1e-10)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    print(f"side-stream solve, {precision}", flush=True)
    Bd = torch.zeros_like(B0)
    torch.cuda._sleep(20_000_000)        # a bounded spin on the current stream
    Bd.copy_(B0)                         # queued behind it
    X, info = helm.solve(F, Bd, tol=1e-10, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    F.close()
    assert info.max_relres <= 1e-10
    assert torch.equal(X, Xref)


def test_release_while_a_solve_is_queued(helm):
    nx, nz, S = 37, 29, 6
    m, w, B = _system(nx, nz, 91, S)
    grid = helm.Grid(nx, nz, 0.04, 0.03)
    own, side = torch.cuda.Stream(), torch.cuda.Stream()
    md = torch.as_tensor(m, device="cuda")
    md2 = torch.as_tensor(m[::-1].copy(), device="cuda")
    B0 = torch.as_tensor(B, device="cuda")
    F = helm.factor(grid, md, w, "fp64", stream=own)
    Xref, _ = helm.solve(F, B0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    torch.cuda._sleep(20_000_000)
    torch.cuda.synchronize()
    t_sleep = time.perf_counter() - t0
    print(f"release while a solve is queued (sleep {t_sleep * 1e3:.1f} ms)", flush=True)
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)
        X, _ = helm.solve(F, B0, stream=side)       # tol 0: queued behind the sleep, no wait
    t0 = time.perf_counter()
    F.close()
    t_close = time.perf_counter() - t0
    F2 = helm.factor(grid, md2, w, "fp64", stream=own)   # takes over F's memory on its stream
    torch.cuda.synchronize()
    F2.close()
    assert torch.equal(X, Xref)
    assert t_close < 0.5 * t_sleep, (t_close, t_sleep)
