"""Python binding of libhelm.so: argument marshalling only.

Every step of the hot path runs in the HIP kernels behind the C ABI declared
in include/helm.h; this module turns torch device tensors into raw pointers
and the current torch stream (or a stream given, ordered after the current
one) into a hipStream_t, and keeps the process's pool of streams for the
serving lanes and the pipeline.  There is no CPU fallback: if the library is
missing or the GPU is absent the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

FP64 = 0
FP32_IR = 1
_PREC = {"fp64": FP64, "fp32_ir": FP32_IR, "fp32": FP32_IR, FP64: FP64, FP32_IR: FP32_IR}

OK, EINVAL, ENOMEM, ESINGULAR, ENOCONV, EDEVICE = 0, -1, -2, -3, -4, -5
_CODES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ESINGULAR: "ESINGULAR", ENOCONV: "ENOCONV", EDEVICE: "EDEVICE"}


class HelmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("hx", ctypes.c_double), ("hz", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int32), ("max_relres", ctypes.c_double), ("bad_block", ctypes.c_int32),
                ("bad_row", ctypes.c_int32), ("solves", ctypes.c_int64)]


@dataclass
class Info:
    ir_iters: int
    max_relres: float
    bad_block: int
    bad_row: int
    solves: int

    @classmethod
    def of(cls, i: _Info) -> "Info":
        return cls(i.ir_iters, i.max_relres, i.bad_block, i.bad_row, i.solves)


@dataclass(frozen=True)
class Grid:
    """n_x x n_z nodes with spacings h_x, h_z; node k = j*n_x + i, j = 0 on top."""
    nx: int
    nz: int
    hx: float
    hz: float

    @property
    def N(self) -> int:
        return self.nx * self.nz

    def c(self) -> _Grid:
        return _Grid(self.nx, self.nz, self.hx, self.hz)

    @classmethod
    def of(cls, w) -> "Grid":
        return cls(int(w.nx), int(w.nz), float(w.hx), float(w.hz))


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def available() -> bool:
    return os.path.exists(LIB_PATH)


def lib():
    """Load libhelm.so (built in-tree by paper_2301_10762_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2301_10762_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    G = ctypes.POINTER(_Grid)
    I = ctypes.POINTER(_Info)
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.helm_factor.argtypes = [G, _vp, f64, ctypes.c_int, _vp, ctypes.POINTER(_vp)]
    L.helm_factor_batch.argtypes = [i32, G, ctypes.POINTER(_vp), ctypes.POINTER(f64), ctypes.c_int, _vp,
                                    ctypes.POINTER(_vp)]
    L.helm_factor_bytes.argtypes = [G, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.helm_factor_destroy.argtypes = [_vp]
    L.helm_factor_destroy.restype = None
    L.helm_solve.argtypes = [_vp, _vp, _vp, i32, i64, f64, _vp, I]
    L.helm_adjoint_solve.argtypes = [_vp, _vp, _vp, i32, i64, f64, _vp, I]
    L.helm_solve_noalloc.argtypes = [_vp, _vp, _vp, i32, i64, f64, _vp, I]
    L.helm_solve_batch.argtypes = [i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                   ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.c_int, f64, _vp, I]
    L.helm_misfit_grad.argtypes = [G, _vp, i32, ctypes.POINTER(f64), _vp, i32, ctypes.POINTER(i32), i32,
                                   ctypes.POINTER(i32), f64, f64, ctypes.c_int, f64, _vp, ctypes.POINTER(f64), _vp, I]
    L.helm_gn_hvp.argtypes = [G, _vp, i32, ctypes.POINTER(f64), i32, ctypes.POINTER(i32), i32, ctypes.POINTER(i32),
                              i32, _vp, f64, f64, ctypes.c_int, f64, _vp, _vp, I]
    L.helm_hess_create.argtypes = [G, _vp, i32, ctypes.POINTER(f64), _vp, i32, ctypes.POINTER(i32), i32,
                                   ctypes.POINTER(i32), f64, f64, ctypes.c_int, f64, _vp, ctypes.POINTER(f64), _vp,
                                   I, ctypes.POINTER(_vp)]
    L.helm_hess_create_at.argtypes = [G, _vp, i32, ctypes.POINTER(f64), _vp, i32, ctypes.POINTER(i32),
                                      ctypes.POINTER(f64), i32, ctypes.POINTER(f64), f64, f64, ctypes.c_int, f64, _vp,
                                      ctypes.POINTER(f64), _vp, I, ctypes.POINTER(_vp)]
    L.helm_point_sources.argtypes = [G, i32, ctypes.POINTER(f64), _vp, i64, _vp]
    L.helm_upper_grad.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(f64), ctypes.POINTER(f64), I]
    L.helm_restrict.argtypes = [G, i32, ctypes.POINTER(f64), ctypes.c_int, _vp, i32, i64, _vp, _vp]
    L.helm_fwi.argtypes = [G, _vp, i32, ctypes.POINTER(f64), _vp, i32, ctypes.POINTER(i32), ctypes.POINTER(f64), i32,
                           ctypes.POINTER(i32), ctypes.POINTER(f64), f64, f64, ctypes.c_int, f64,
                           ctypes.POINTER(_LbfgsOpts), _vp, ctypes.POINTER(f64), ctypes.POINTER(_FwiInfo)]
    L.helm_hess_apply.argtypes = [_vp, i32, _vp, _vp, _vp, I]
    L.helm_hess_pcg.argtypes = [_vp, _vp, _vp, f64, f64, f64, i32, _vp, ctypes.POINTER(i32), ctypes.POINTER(f64), I]
    L.helm_hess_pcg_batch.argtypes = [i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), f64, f64,
                                      f64, i32, _vp, ctypes.POINTER(i32), ctypes.POINTER(f64), ctypes.POINTER(i32), I]
    L.helm_hess_destroy.argtypes = [_vp]
    L.helm_hess_destroy.restype = None
    L.helm_gamma_solve.argtypes = [G, f64, f64, i32, _vp, _vp, _vp]
    L.helm_residual.argtypes = [G, _vp, f64, ctypes.c_int, _vp, _vp, _vp, i32, i64, _vp, _vp]
    L.helm_tile_inverse.argtypes = [i32, i32, ctypes.c_int, _vp, _vp, _vp]
    L.helm_set_tile_pivoting.argtypes = [ctypes.c_int]
    L.helm_set_tile_pivoting.restype = None
    L.helm_set_cache_limit.argtypes = [ctypes.c_size_t]
    L.helm_set_cache_limit.restype = ctypes.c_size_t
    L.helm_mfma_probe.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp]
    L.helm_kernel_timing.argtypes = [ctypes.c_int]
    L.helm_kernel_timing.restype = None
    L.helm_kernel_time.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.helm_kernel_time.restype = ctypes.c_int
    L.helm_counter.argtypes = [ctypes.c_int]
    L.helm_counter.restype = ctypes.c_int64
    L.helm_last_error.restype = ctypes.c_char_p
    for name in ("helm_factor", "helm_factor_batch", "helm_factor_bytes", "helm_solve", "helm_adjoint_solve",
                 "helm_solve_batch", "helm_misfit_grad", "helm_gn_hvp", "helm_residual", "helm_tile_inverse",
                 "helm_mfma_probe", "helm_hess_create", "helm_hess_apply", "helm_hess_pcg", "helm_gamma_solve",
                 "helm_hess_create_at", "helm_upper_grad", "helm_restrict", "helm_fwi",
                 "helm_point_sources", "helm_hess_pcg_batch"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise HelmError(rc, lib().helm_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libhelm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(stream=None):
    """Handle of the stream a call runs on: `stream`, else the current one.
    A stream other than the current one first waits for the work already
    queued on the current stream, in whose order the call's inputs were
    written and its outputs allocated."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return _vp(cur.cuda_stream)
    stream.wait_stream(cur)
    return _vp(stream.cuda_stream)


_POOL = {}   # (device, key) -> stream, made once per process


def pooled_stream(key):
    """The process's stream for `key` on the current device, made on first
    use; the serving lanes and the pipeline take their streams from here.
    * torch's caching allocator keeps a block freed on a stream for later
      allocations on that same stream: runs that made new streams each time
      would leave every earlier run's results cached where no later run can
      use them, until the device is full.
    * The runtime maps streams onto a few hardware queues per process as
      they come into use; a second set of new streams can land on one
      shared queue, and the work meant to overlap then runs in turn.
    Users of one key at the same time (threads) share its stream: their
    work is ordered, results are unchanged."""
    torch = _torch()
    k = (torch.cuda.current_device(), key)
    s = _POOL.get(k)
    if s is None:
        s = _POOL[k] = torch.cuda.Stream()
    return s


def _written_on(stream, *outs):
    """Outputs allocated here (on the current stream) and written on another
    `stream` by a call that may return before its kernels end: the caching
    allocator must not reuse their memory until that stream is done."""
    torch = _torch()
    if stream is not None and stream != torch.cuda.current_stream():
        for t in outs:
            t.record_stream(stream)


def _ptr(t) -> _vp:
    return _vp(t.data_ptr())


def _dev_f64(x, n=None):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


def _dev_c128(x):
    torch = _torch()
    t = torch.as_tensor(x, device="cuda")
    if t.dtype != torch.complex128:
        t = t.to(torch.complex128)
    return t.contiguous()


def _src_arg(sources):
    """(count, node pointer or None, point pointer or None, keep-alive) for
    sources given as node indices or as an [S][2] float array of points."""
    a = np.asarray(sources)
    if a.dtype.kind == "f":
        pts = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 2)
        return len(pts), None, pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), pts
    arr, ptr = _i32(sources)
    return len(arr), ptr, None, arr


def _i32(seq):
    a = np.ascontiguousarray(np.asarray(seq, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def counters() -> dict:
    L = lib()
    return {"launches": int(L.helm_counter(0)), "solves": int(L.helm_counter(1)),
            "cached_bytes": int(L.helm_counter(4))}


KERNEL_KINDS = {"factor_step": 0, "factor_init": 1, "sweep": 2}


def kernel_timing(enable: bool):
    """Bracket every run of back-to-back hot-kernel launches with HIP events."""
    lib().helm_kernel_timing(int(enable))


def kernel_time(kind: str):
    """(total ms, timed launches) of a kernel kind since kernel_timing(True)."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().helm_kernel_time(KERNEL_KINDS[kind], ctypes.byref(ms), ctypes.byref(cnt)))
    return float(ms.value), int(cnt.value)


def factor_bytes(grid: Grid, precision="fp64") -> int:
    out = ctypes.c_size_t(0)
    _check(lib().helm_factor_bytes(ctypes.byref(grid.c()), _PREC[precision], ctypes.byref(out)))
    return int(out.value)


class Factor:
    """Device factorisation of A(m, w); owns HBM until close()."""

    def __init__(self, handle: int, grid: Grid, omega: float, precision: int):
        self._h = _vp(handle)
        self.grid = grid
        self.omega = float(omega)
        self.precision = precision

    @property
    def handle(self) -> _vp:
        if not self._h:
            raise RuntimeError("factor already destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().helm_factor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, B, tol: float = 0.0, stream=None):
        return solve(self, B, tol, stream)

    def adjoint_solve(self, R, tol: float = 0.0, stream=None):
        return adjoint_solve(self, R, tol, stream)


def factor(grid: Grid, m, omega: float, precision="fp64", stream=None) -> Factor:
    """Factor A(m, w) on the GPU (block-tridiagonal LU, one block per grid row)."""
    md = _dev_f64(m, grid.N)
    h = _vp()
    _check(lib().helm_factor(ctypes.byref(grid.c()), _ptr(md), float(omega), _PREC[precision], _stream(stream),
                             ctypes.byref(h)))
    return Factor(h.value, grid, omega, _PREC[precision])


def factor_batch(grids, ms, omegas, precision="fp64", stream=None) -> list:
    """Factor several systems with their block chains sharing kernel launches."""
    n = len(omegas)
    grids = list(grids) if not isinstance(grids, Grid) else [grids] * n
    mds = [_dev_f64(m, g.N) for m, g in zip(ms, grids)]
    garr = (_Grid * n)(*[g.c() for g in grids])
    marr = (_vp * n)(*[md.data_ptr() for md in mds])
    warr = (ctypes.c_double * n)(*[float(w) for w in omegas])
    outs = (_vp * n)()
    _check(lib().helm_factor_batch(n, garr, marr, warr, _PREC[precision], _stream(stream), outs))
    return [Factor(outs[c], grids[c], omegas[c], _PREC[precision]) for c in range(n)]


def _rhs(F: Factor, B):
    B = _dev_c128(B)
    if B.dim() == 1:
        B = B.unsqueeze(0)
    if B.shape[-1] != F.grid.N:
        raise ValueError("right-hand sides must be [S][nx*nz]")
    return B


def solve(F: Factor, B, tol: float = 0.0, stream=None):
    """X = A^{-1} B (rows of B are right-hand sides).  Returns (X, Info)."""
    torch = _torch()
    B = _rhs(F, B)
    X = torch.empty_like(B)
    info = _Info()
    _check(lib().helm_solve(F.handle, _ptr(B), _ptr(X), B.shape[0], F.grid.N, float(tol), _stream(stream),
                            ctypes.byref(info)))
    _written_on(stream, X)
    return X, Info.of(info)


def solve_noalloc(F: Factor, B, X, tol: float = 0.0, stream=None):
    """X = A^{-1} B into the caller's X with no device allocation: the
    call's scratch comes from the library's fixed per-device region
    (helm_solve_noalloc).  B and X are complex128 [S][nx*nz] device tensors.
    Returns Info."""
    if B.dtype != X.dtype or B.shape != X.shape or B.dim() != 2 or B.shape[-1] != F.grid.N:
        raise ValueError("B and X must be [S][nx*nz] tensors of the same shape")
    if not (B.is_contiguous() and X.is_contiguous()) or str(B.dtype) != "torch.complex128":
        raise ValueError("B and X must be contiguous complex128")
    info = _Info()
    _check(lib().helm_solve_noalloc(F.handle, _ptr(B), _ptr(X), B.shape[0], F.grid.N, float(tol), _stream(stream),
                                    ctypes.byref(info)))
    return Info.of(info)


def adjoint_solve(F: Factor, R, tol: float = 0.0, stream=None):
    """L = A^{-*} R, the conjugate-transpose solve with the same factors."""
    torch = _torch()
    R = _rhs(F, R)
    L = torch.empty_like(R)
    info = _Info()
    _check(lib().helm_adjoint_solve(F.handle, _ptr(R), _ptr(L), R.shape[0], F.grid.N, float(tol), _stream(stream),
                                    ctypes.byref(info)))
    _written_on(stream, L)
    return L, Info.of(info)


def solve_batch(Fs, Bs, adjoint: bool = False, tol: float = 0.0, stream=None, out=None):
    """Solve with several factors at once; sweeps share kernel launches."""
    torch = _torch()
    n = len(Fs)
    Bs = [_rhs(F, B) for F, B in zip(Fs, Bs)]
    Xs = out if out is not None else [torch.empty_like(B) for B in Bs]
    harr = (_vp * n)(*[F.handle.value for F in Fs])
    barr = (_vp * n)(*[B.data_ptr() for B in Bs])
    xarr = (_vp * n)(*[X.data_ptr() for X in Xs])
    sarr = (ctypes.c_int32 * n)(*[B.shape[0] for B in Bs])
    larr = (ctypes.c_int64 * n)(*[F.grid.N for F in Fs])
    infos = (_Info * n)()
    _check(lib().helm_solve_batch(n, harr, barr, xarr, sarr, larr, int(adjoint), float(tol), _stream(stream), infos))
    if out is None:
        _written_on(stream, *Xs)
    return Xs, [Info.of(infos[c]) for c in range(n)]


def misfit_grad(grid: Grid, m, omegas, d_obs, sources, receivers, alpha: float = 0.0, mu: float = 0.0,
                precision="fp64", tol: float = 0.0, stream=None, grad_out=None):
    """phi and grad phi by the adjoint-state method (appendix "Gradient of phi",
    Algorithm 3).  d_obs: complex [n_omega][S][Nr]."""
    torch = _torch()
    md = _dev_f64(m, grid.N)
    n_omega = len(omegas)
    src, psrc = _i32(sources)
    rec, prec = _i32(receivers)
    dd = _dev_c128(d_obs)
    if tuple(dd.shape) != (n_omega, len(src), len(rec)):
        raise ValueError("d_obs must be [n_omega][S][Nr]")
    warr = (ctypes.c_double * n_omega)(*[float(w) for w in omegas])
    g = grad_out if grad_out is not None else torch.empty(grid.N, dtype=torch.float64, device="cuda")
    phi = ctypes.c_double(0.0)
    info = _Info()
    _check(lib().helm_misfit_grad(ctypes.byref(grid.c()), _ptr(md), n_omega, warr, _ptr(dd), len(src), psrc,
                                  len(rec), prec, float(alpha), float(mu), _PREC[precision], float(tol),
                                  _stream(stream), ctypes.byref(phi), _ptr(g), ctypes.byref(info)))
    if grad_out is None:
        _written_on(stream, g)
    return float(phi.value), g, Info.of(info)


def gn_hvp(grid: Grid, m, omegas, sources, receivers, directions, alpha: float = 0.0, mu: float = 0.0,
           precision="fp64", tol: float = 0.0, stream=None):
    """(H^(1) + Gamma) mt for each direction (rows of `directions`)."""
    torch = _torch()
    md = _dev_f64(m, grid.N)
    mt = _dev_f64(directions)
    mt = mt.reshape(-1, grid.N).contiguous()
    n_omega = len(omegas)
    src, psrc = _i32(sources)
    rec, prec = _i32(receivers)
    warr = (ctypes.c_double * n_omega)(*[float(w) for w in omegas])
    hv = torch.empty_like(mt)
    info = _Info()
    _check(lib().helm_gn_hvp(ctypes.byref(grid.c()), _ptr(md), n_omega, warr, len(src), psrc, len(rec), prec,
                             mt.shape[0], _ptr(mt), float(alpha), float(mu), _PREC[precision], float(tol),
                             _stream(stream), _ptr(hv), ctypes.byref(info)))
    _written_on(stream, hv)
    return hv, Info.of(info)


class _LbfgsOpts(ctypes.Structure):
    _fields_ = [("memory", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("max_evals", ctypes.c_int32),
                ("gtol", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("first_change", ctypes.c_double)]


class _FwiInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("evals", ctypes.c_int32), ("status", ctypes.c_int32),
                ("phi0", ctypes.c_double), ("phi", ctypes.c_double), ("gnorm0", ctypes.c_double),
                ("gnorm", ctypes.c_double), ("solves", ctypes.c_int64)]


_FWI_STATUS = {0: "converged", 1: "max_iters", 2: "line_search"}


def fwi(grid: Grid, m0, omegas, d_obs, sources, receivers, alpha: float = 0.0, mu: float = 0.0, precision="fp64",
        tol: float = 0.0, memory: int = 5, max_iters: int = 50, gtol: float = 1e-6, c1: float = 1e-4,
        c2: float = 0.9, max_evals: int = 20, first_change: float = 0.01, stream=None):
    """Lower-level FWI by L-BFGS with a strong-Wolfe line search (helm_fwi).
    receivers: node indices or [Nr][2] sensor points.  Returns (m, info)
    with info = {iterations, evals, status, phi0, phi, gnorm0, gnorm,
    solves, history}."""
    m = _dev_f64(m0, grid.N).clone()
    n_omega = len(omegas)
    n_src, psrc, psxz, _keep = _src_arg(sources)
    rarr = np.asarray(receivers)
    if rarr.dtype.kind == "f":
        rec = np.ascontiguousarray(rarr, dtype=np.float64).reshape(-1, 2)
        prec_i, prec_xz = None, rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    else:
        rec, prec_i = _i32(receivers)
        prec_xz = None
    dd = _dev_c128(d_obs)
    if tuple(dd.shape) != (n_omega, n_src, len(rec)):
        raise ValueError("d_obs must be [n_omega][S][Nr]")
    warr = (ctypes.c_double * n_omega)(*[float(w) for w in omegas])
    opts = _LbfgsOpts(int(memory), int(max_iters), int(max_evals), float(gtol), float(c1), float(c2),
                      float(first_change))
    hist = (ctypes.c_double * (int(max_iters) + 1))()
    info = _FwiInfo()
    _check(lib().helm_fwi(ctypes.byref(grid.c()), _ptr(m), n_omega, warr, _ptr(dd), n_src, psrc, psxz, len(rec),
                          prec_i, prec_xz, float(alpha), float(mu), _PREC[precision], float(tol), ctypes.byref(opts),
                          _stream(stream), hist, ctypes.byref(info)))
    out = {k: getattr(info, k) for k, _ in _FwiInfo._fields_}
    out["status"] = _FWI_STATUS.get(info.status, info.status)
    out["history"] = [hist[i] for i in range(info.iterations + 1)]
    return m, out


def fwi_continuation(grid: Grid, m0, groups, omegas, d_obs, sources, receivers, **kw):
    """FWI over frequency groups in turn, each started from the previous
    result (the lower level of the bilevel frequency continuation, App.
    "Bilevel Frequency Continuation").  groups: lists of frequency indices
    into omegas / d_obs.  Returns (m, [info per group])."""
    torch = _torch()
    dd = _dev_c128(d_obs)
    m = _dev_f64(m0, grid.N)
    infos = []
    for grp in groups:
        idx = [int(i) for i in grp]
        m, info = fwi(grid, m, [omegas[i] for i in idx], dd[torch.as_tensor(idx, device=dd.device)].contiguous(),
                      sources, receivers, **kw)
        infos.append(info)
    return m, infos


class Hessian:
    """Lower-level state at one model for products with the Hessian of phi
    (helm_hess_create): with d_obs ([n_omega][S][Nr] complex) the full
    H = H^(1) + H^(2) + Gamma, without it the Gauss-Newton H^(1) + Gamma.
    with_grad=True also returns phi and grad phi (data required).
    receivers: node indices, or an [Nr][2] float array of sensor points
    (x, z) with the sliding-cubic restriction (helm_hess_create_at)."""

    def __init__(self, grid: Grid, m, omegas, sources, receivers, d_obs=None, alpha: float = 0.0, mu: float = 0.0,
                 precision="fp64", tol: float = 0.0, stream=None, with_grad: bool = False):
        torch = _torch()
        self.grid = grid
        self.h = None
        md = _dev_f64(m, grid.N)
        n_omega = len(omegas)
        n_src, psrc, psxz, _keep = _src_arg(sources)
        rarr = np.asarray(receivers)
        self.at_points = rarr.dtype.kind == "f" or psxz is not None
        if rarr.dtype.kind == "f":
            rec = np.ascontiguousarray(rarr, dtype=np.float64).reshape(-1, 2)
            prec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        elif self.at_points:
            # point sources with node receivers: the receivers as points
            nodes = np.asarray(receivers, dtype=np.int64)
            rec = np.ascontiguousarray(np.column_stack([(nodes % grid.nx) * grid.hx, (nodes // grid.nx) * grid.hz]))
            prec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            rec, prec = _i32(receivers)
        self.n_omega, self.S, self.Nr = n_omega, n_src, len(rec)
        dd = None
        if d_obs is not None:
            dd = _dev_c128(d_obs)
            if tuple(dd.shape) != (n_omega, n_src, len(rec)):
                raise ValueError("d_obs must be [n_omega][S][Nr]")
        elif with_grad:
            raise ValueError("phi and grad need data")
        warr = (ctypes.c_double * n_omega)(*[float(w) for w in omegas])
        phi = ctypes.c_double(0.0)
        self.grad = torch.empty(grid.N, dtype=torch.float64, device="cuda") if with_grad else None
        info = _Info()
        h = ctypes.c_void_p()
        if self.at_points:
            create = lambda *a: lib().helm_hess_create_at(*a[:7], psxz, *a[7:])     # noqa: E731
        else:
            create = lib().helm_hess_create
        _check(create(ctypes.byref(grid.c()), _ptr(md), n_omega, warr,
                                      _ptr(dd) if dd is not None else None, n_src, psrc, len(rec), prec,
                                      float(alpha), float(mu), _PREC[precision], float(tol), _stream(stream),
                                      ctypes.byref(phi) if with_grad else None,
                                      _ptr(self.grad) if with_grad else None, ctypes.byref(info), ctypes.byref(h)))
        self.h = h
        self.phi = float(phi.value) if with_grad else None
        self.info = Info.of(info)

    def apply(self, directions, stream=None):
        """H mt for each row of `directions` ([n_dir][N] or [N])."""
        torch = _torch()
        mt = _dev_f64(directions).reshape(-1, self.grid.N).contiguous()
        hv = torch.empty_like(mt)
        info = _Info()
        _check(lib().helm_hess_apply(self.h, mt.shape[0], _ptr(mt), _ptr(hv), _stream(stream), ctypes.byref(info)))
        _written_on(stream, hv)
        return hv, Info.of(info)

    def pcg(self, b, x0=None, prec_alpha: float = 0.0, prec_mu: float = 0.0, rtol: float = 1e-6,
            maxit: int = 1000, stream=None, strict: bool = True):
        """PCG for H x = b with P2 = Gamma(prec_alpha, prec_mu) (none when
        prec_mu <= 0); start vector all ones unless x0 is given.  Returns
        (x, iterations, final ||r|| / ||r0||, info).  strict=False returns
        the last iterate instead of raising when the tolerance is not met
        within maxit."""
        torch = _torch()
        bd = _dev_f64(b, self.grid.N).contiguous()
        x = (torch.ones(self.grid.N, dtype=torch.float64, device="cuda") if x0 is None
             else _dev_f64(x0, self.grid.N).clone())
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        info = _Info()
        rc = lib().helm_hess_pcg(self.h, _ptr(bd), _ptr(x), float(prec_alpha), float(prec_mu), float(rtol),
                                 int(maxit), _stream(stream), ctypes.byref(it), ctypes.byref(rel), ctypes.byref(info))
        if rc != OK and (strict or rc != ENOCONV or int(it.value) < int(maxit)):
            _check(rc)
        return x, int(it.value), float(rel.value), Info.of(info)

    def upper_grad(self, rho, ddata, stream=None):
        """dpsi/dp ([Nr][2], x and z) and dpsi/dalpha for this training
        model (helm_upper_grad).  ddata: complex [n_omega][S][Nr][2], the
        sensor-coordinate derivatives of the training wavefield."""
        rd = _dev_f64(rho, self.grid.N).contiguous()
        dd = _dev_c128(ddata)
        if tuple(dd.shape) != (self.n_omega, self.S, self.Nr, 2):
            raise ValueError("ddata must be [n_omega][S][Nr][2]")
        dp = np.zeros((self.Nr, 2))
        da = ctypes.c_double(0.0)
        info = _Info()
        _check(lib().helm_upper_grad(self.h, _ptr(rd), _ptr(dd), _stream(stream),
                                     dp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(da),
                                     ctypes.byref(info)))
        return dp, float(da.value), Info.of(info)

    def close(self):
        if self.h:
            lib().helm_hess_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def point_sources(grid: Grid, positions, stream=None):
    """Right-hand sides of point sources between nodes ([S][2] points):
    helm_point_sources.  Returns complex [S][N]."""
    torch = _torch()
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    B = torch.empty((len(pos), grid.N), dtype=torch.complex128, device="cuda")
    _check(lib().helm_point_sources(ctypes.byref(grid.c()), len(pos),
                                    pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(B), grid.N,
                                    _stream(stream)))
    _written_on(stream, B)
    return B


def restrict(grid: Grid, positions, U, deriv: int = 0, stream=None):
    """R(P) U (deriv 0) or d/dx (1), d/dz (2) of it for sensors at points
    ([Nr][2]) and fields U ([S][N] complex); returns [S][Nr] complex."""
    torch = _torch()
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    Ud = _dev_c128(U).reshape(-1, grid.N).contiguous()
    out = torch.empty((Ud.shape[0], len(pos)), dtype=torch.complex128, device="cuda")
    _check(lib().helm_restrict(ctypes.byref(grid.c()), len(pos), pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               int(deriv), _ptr(Ud), Ud.shape[0], grid.N, _ptr(out), _stream(stream)))
    _written_on(stream, out)
    return out


_PCG_STATUS = {0: "converged", 1: "max_iters", 2: "indefinite"}


def pcg_batch(contexts, bs, x0s=None, prec_alpha: float = 0.0, prec_mu: float = 0.0, rtol: float = 1e-6,
              maxit: int = 1000, stream=None):
    """PCG for several Hessian systems in lockstep (helm_hess_pcg_batch):
    contexts[c] x_c = bs[c].  Returns ([x_c], [iterations], [relres],
    [status], [Info])."""
    torch = _torch()
    K = len(contexts)
    bd = [_dev_f64(b, H.grid.N).contiguous() for b, H in zip(bs, contexts)]
    xs = [torch.ones(H.grid.N, dtype=torch.float64, device="cuda") if x0s is None
          else _dev_f64(x0s[c], H.grid.N).clone() for c, H in enumerate(contexts)]
    harr = (_vp * K)(*[H.h for H in contexts])
    barr = (_vp * K)(*[b.data_ptr() for b in bd])
    xarr = (_vp * K)(*[x.data_ptr() for x in xs])
    it = (ctypes.c_int32 * K)()
    rr = (ctypes.c_double * K)()
    stt = (ctypes.c_int32 * K)()
    infos = (_Info * K)()
    _check(lib().helm_hess_pcg_batch(K, harr, barr, xarr, float(prec_alpha), float(prec_mu), float(rtol), int(maxit),
                                     _stream(stream), it, rr, stt, infos))
    return (xs, [int(v) for v in it], [float(v) for v in rr], [_PCG_STATUS.get(v, v) for v in stt],
            [Info.of(infos[c]) for c in range(K)])


def gamma_solve(grid: Grid, alpha: float, mu: float, Y, stream=None):
    """Gamma(alpha, mu)^{-1} Y for each row of Y (the P2 preconditioner)."""
    torch = _torch()
    Yd = _dev_f64(Y).reshape(-1, grid.N).contiguous()
    X = torch.empty_like(Yd)
    _check(lib().helm_gamma_solve(ctypes.byref(grid.c()), float(alpha), float(mu), Yd.shape[0], _ptr(Yd), _ptr(X),
                                  _stream(stream)))
    _written_on(stream, X)
    return X


def residual(grid: Grid, m, omega: float, B, X, adjoint: bool = False, stream=None):
    """(r = B - A X, per-column [||r||^2, ||B||^2]) in FP64 on the GPU."""
    torch = _torch()
    md = _dev_f64(m, grid.N)
    B = _dev_c128(B).reshape(-1, grid.N).contiguous()
    X = _dev_c128(X).reshape(-1, grid.N).contiguous()
    r = torch.empty_like(B)
    norms = torch.empty(B.shape[0], 2, dtype=torch.float64, device="cuda")
    _check(lib().helm_residual(ctypes.byref(grid.c()), _ptr(md), float(omega), int(adjoint), _ptr(B), _ptr(X),
                               _ptr(r), B.shape[0], grid.N, _ptr(norms), _stream(stream)))
    _written_on(stream, r, norms)
    return r, norms


def tile_inverse(A, pivot: bool = True):
    """Inverse of each kb x kb complex128 tile (kb = 16 or 32) by the factorisation's Gauss-Jordan."""
    torch = _torch()
    A = _dev_c128(A)
    count, kb = A.shape[0], A.shape[1]
    T = torch.empty_like(A)
    _check(lib().helm_tile_inverse(count, kb, int(pivot), _ptr(A), _ptr(T), _stream()))
    return T


def set_tile_pivoting(always: bool):
    """Always invert diagonal tiles with partial pivoting (process-wide)."""
    lib().helm_set_tile_pivoting(int(always))


def set_cache_limit(nbytes: int) -> int:
    """Bytes of freed device blocks the library keeps for reuse (0 empties
    the cache); returns the previous limit."""
    return int(lib().helm_set_cache_limit(int(nbytes)))


def mfma_probe(prec: int, A, B):
    torch = _torch()
    A = _dev_f64(A, 64)
    B = _dev_f64(B, 64)
    D = torch.zeros(256, dtype=torch.float64, device="cuda")
    _check(lib().helm_mfma_probe(int(prec), _ptr(A), _ptr(B), _ptr(D), _stream()))
    return D.reshape(16, 16)
