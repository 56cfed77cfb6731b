"""Seeded synthetic inputs for the Helmholtz hot path.

This module only *generates* inputs: earth models m = 1/c^2, frequencies,
source/receiver node lists, Gauss-Newton directions and serving request
streams.  It holds none of the method's arithmetic (no operator, no solve, no
misfit) and imports nothing else from this package, so that both the CPU
oracle's tests and the GPU path can draw the same inputs from it.

Grid convention: an n_x x n_z node grid, node k = j*n_x + i, x_i = i*h_x,
z_j = j*h_z, j = 0 is the top (surface) row.

The paper's experiments use smoothed Marmousi slices on a 25 m grid with
velocities of 1.5-4.5 km/s and frequencies up to 6 Hz (Section 4).  That data
is not available here; the layered-plus-random-field family below stands in
for it with the same spacing, velocity range and frequency band.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

H_KM = 0.025          # 25 m grid spacing of the paper's Marmousi runs (Section 4)
C_MIN, C_MAX = 1.5, 4.5  # km/s


# ----------------------------------------------------------------------------
# earth models
# ----------------------------------------------------------------------------

def blob_model(n: int = 33, amplitude: float = 0.3, width: float = 0.1) -> np.ndarray:
    """Unit square, c = 1 + amplitude*exp(-|x-(.5,.5)|^2/(2 width^2)); returns m = 1/c^2."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Z = np.meshgrid(x, x, indexing="xy")          # [j][i]
    c = 1.0 + amplitude * np.exp(-((X - 0.5) ** 2 + (Z - 0.5) ** 2) / (2 * width ** 2))
    return np.ascontiguousarray((1.0 / c ** 2).reshape(-1))


def gaussian_random_field(shape, rng: np.random.Generator, corr_cells: float) -> np.ndarray:
    """White noise filtered in Fourier space by a Gaussian kernel of the given
    correlation length (in cells), normalised to zero mean and unit std."""
    nz, nx = shape
    w = rng.standard_normal((nz, nx))
    kz = np.fft.fftfreq(nz)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi * corr_cells) ** 2 * (kx ** 2 + kz ** 2))
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    g -= g.mean()
    s = g.std()
    return g / s if s > 0 else g


def layered_velocity(nx: int, nz: int, seed: int, h: float = H_KM,
                     n_interfaces: int = 6, grf_std: float = 0.05,
                     grf_corr_cells: float = 10.0) -> np.ndarray:
    """Layered velocity c[j][i] (km/s): 6 smooth random interfaces, 7 layer
    speeds sorted ascending in [1.5, 4.5], times (1 + 5% Gaussian random field
    of correlation length 10 cells), clipped to [1.5, 4.5]."""
    rng = np.random.default_rng(seed)
    Lx = (nx - 1) * h
    Lz = (nz - 1) * h
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    zbar = np.sort(rng.uniform(0.05 * Lz, 0.95 * Lz, n_interfaces))
    amp = rng.uniform(-0.03 * Lz, 0.03 * Lz, (n_interfaces, 3))
    phase = rng.uniform(0.0, 2 * math.pi, (n_interfaces, 3))
    speeds = np.sort(rng.uniform(C_MIN, C_MAX, n_interfaces + 1))
    surf = np.empty((n_interfaces, nx))
    for a in range(n_interfaces):
        s = np.full(nx, zbar[a])
        for q in range(3):
            s += amp[a, q] * np.sin(2 * math.pi * (q + 1) * x / max(Lx, 1e-30) + phase[a, q])
        surf[a] = s
    Z = z[:, None]
    layer = np.zeros((nz, nx), dtype=np.int64)
    for a in range(n_interfaces):
        layer += (Z > surf[a][None, :]).astype(np.int64)
    c = speeds[layer]
    g = gaussian_random_field((nz, nx), rng, grf_corr_cells)
    c = np.clip(c * (1.0 + grf_std * g), C_MIN, C_MAX)
    return c


def smooth_velocity(c: np.ndarray, corr_cells: float) -> np.ndarray:
    """Gaussian smoothing of a velocity field (edge-padded FFT filter)."""
    nz, nx = c.shape
    p = int(math.ceil(3 * corr_cells))
    cp = np.pad(c, p, mode="edge")
    kz = np.fft.fftfreq(cp.shape[0])[:, None]
    kx = np.fft.fftfreq(cp.shape[1])[None, :]
    filt = np.exp(-2.0 * (math.pi * corr_cells) ** 2 * (kx ** 2 + kz ** 2))
    cs = np.real(np.fft.ifft2(np.fft.fft2(cp) * filt))
    return cs[p:p + nz, p:p + nx]


def layered_model(n: int, seed: int, h: float = H_KM) -> np.ndarray:
    """m = 1/c^2 (s^2/km^2) of the layered family on an n x n grid, flat [j*n + i]."""
    c = layered_velocity(n, n, seed, h)
    return np.ascontiguousarray((1.0 / c ** 2).reshape(-1))


def layered_pair(n: int, seed: int, h: float = H_KM, smooth_cells: float = 20.0):
    """(m_true, m_start): a layered ground truth and a smoothed starting model
    (the usual FWI set-up: data come from m_true, the misfit is evaluated at m_start)."""
    c = layered_velocity(n, n, seed, h)
    cs = np.clip(smooth_velocity(c, smooth_cells), C_MIN, C_MAX)
    return (np.ascontiguousarray((1.0 / c ** 2).reshape(-1)),
            np.ascontiguousarray((1.0 / cs ** 2).reshape(-1)))


# ----------------------------------------------------------------------------
# frequencies and acquisition
# ----------------------------------------------------------------------------

def omega_from_ppw(ppw: float, c_min: float, h: float) -> float:
    """Angular frequency giving `ppw` points per wavelength at speed c_min."""
    return 2.0 * math.pi * c_min / (ppw * h)


def line_nodes(nx: int, j: int, i_list) -> np.ndarray:
    return np.asarray([j * nx + int(i) for i in i_list], dtype=np.int32)


def surface_sources(n: int, count: int, depth: int = 2, margin=None) -> np.ndarray:
    lo, hi = margin if margin is not None else (5, n - 6)
    i = np.round(np.linspace(lo, hi, count)).astype(int)
    return line_nodes(n, depth, i)


def surface_receivers(n: int, count: int, step: int = 2) -> np.ndarray:
    return line_nodes(n, 0, [step * q for q in range(count)])


@dataclass
class Workload:
    """One configuration of the hot path: grid, models, frequencies, acquisition."""
    name: str
    nx: int
    nz: int
    hx: float
    hz: float
    m: np.ndarray            # model at which phi / grad are evaluated
    m_true: np.ndarray       # model that generates the synthetic data
    omegas: list
    sources: np.ndarray      # int32 node indices
    receivers: np.ndarray    # int32 node indices
    directions: list = field(default_factory=list)   # Gauss-Newton directions

    @property
    def N(self):
        return self.nx * self.nz


def gn_directions(nx: int, nz: int, count: int, seed: int, norm: float,
                  corr_cells: float = 10.0) -> list:
    """Smoothed N(0,1) directions, each scaled to Euclidean norm `norm`."""
    rng = np.random.default_rng(10_000 + seed)
    out = []
    for _ in range(count):
        g = gaussian_random_field((nz, nx), rng, corr_cells).reshape(-1)
        out.append(np.ascontiguousarray(g * (norm / np.linalg.norm(g))))
    return out


def config_c1() -> Workload:
    """33 x 33 unit square, blob c = 1 + 0.3 bump (width 0.1), one frequency at
    >= 10 points per wavelength (omega = 2*pi*3, PPW = 32/3 at c = 1), 4 sources
    and 16 receivers on the top row (never coinciding)."""
    n = 33
    h = 1.0 / (n - 1)
    m = blob_model(n, 0.30)
    m_true = blob_model(n, 0.35)
    src = line_nodes(n, 0, [4, 12, 20, 28])
    rec = line_nodes(n, 0, list(range(1, 32, 2)))
    return Workload("c1_blob_33", n, n, h, h, m, m_true, [2 * math.pi * 3.0], src, rec)


def config_layered(n: int, ppws, n_src: int, n_rec: int, seed: int, name: str,
                   n_dirs: int = 0) -> Workload:
    m_true, m = layered_pair(n, seed)
    omegas = [omega_from_ppw(p, C_MIN, H_KM) for p in ppws]
    src = surface_sources(n, n_src, depth=2, margin=(5, n - 6) if n < 300 else (4, n - 5))
    rec = surface_receivers(n, n_rec)
    dirs = gn_directions(n, n, n_dirs, seed, float(np.linalg.norm(m))) if n_dirs else []
    return Workload(name, n, n, H_KM, H_KM, m, m_true, omegas, src, rec, dirs)


def config_c2(seed: int = 0) -> Workload:
    """201^2 layered model, 3 frequencies (20, 14, 10 PPW), 30 sources, 100 receivers."""
    return config_layered(201, [20.0, 14.0, 10.0], 30, 100, seed, "c2_layered_201")


def config_c3(seed: int = 1) -> Workload:
    """401^2 layered model, 5 frequencies (1.5-6 Hz), 64 sources, 200 receivers."""
    return config_layered(401, [40.0, 80.0 / 3.0, 20.0, 40.0 / 3.0, 10.0], 64, 200, seed,
                          "c3_layered_401")


def config_c4(seed: int = 2) -> Workload:
    """201^2, 4 frequencies (20, 15, 12, 10 PPW), 32 sources, 100 receivers, 8 GN directions."""
    return config_layered(201, [20.0, 15.0, 12.0, 10.0], 32, 100, seed, "c4_layered_201", 8)


def small_layered(n: int, seed: int, n_src: int, n_rec: int, ppws=(10.0,), n_dirs: int = 0,
                  h: float = H_KM) -> Workload:
    """A shrunken member of the layered family, for tests."""
    m_true, m = layered_pair(n, seed, h)
    omegas = [omega_from_ppw(p, C_MIN, h) for p in ppws]
    src = surface_sources(n, n_src, depth=2, margin=(1, n - 2))
    rec = line_nodes(n, 0, np.round(np.linspace(0, n - 1, n_rec)).astype(int))
    dirs = gn_directions(n, n, n_dirs, seed, float(np.linalg.norm(m))) if n_dirs else []
    return Workload(f"small_{n}", n, n, h, h, m, m_true, list(omegas), src, rec, dirs)


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    t_arrival: float      # seconds from stream start
    n: int
    ppw: float
    n_src: int
    seed: int


def serving_stream(count: int, rate_hz: float = 200.0, seed: int = 0,
                   sizes=(101, 201, 301, 401), ppw_range=(8.0, 15.0),
                   src_range=(8, 128)) -> list:
    """Poisson arrivals; n uniform over `sizes`, PPW uniform in `ppw_range`,
    source count uniform in `src_range`; each request has its own model seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate_hz)
        out.append(Request(r, t, int(rng.choice(sizes)), float(rng.uniform(*ppw_range)),
                           int(rng.integers(src_range[0], src_range[1] + 1)), 1000 + r))
    return out


def request_inputs(req: Request):
    """Model, omega and source nodes of one serving request."""
    m = layered_model(req.n, req.seed)
    omega = omega_from_ppw(req.ppw, C_MIN, H_KM)
    src = surface_sources(req.n, req.n_src, depth=2, margin=(1, req.n - 2))
    return m, omega, src


def point_sources(N: int, nodes, dtype=np.complex128) -> np.ndarray:
    """Column-major N x S block of unit vectors e_s (S = len(nodes)), as [S][N]."""
    B = np.zeros((len(nodes), N), dtype=dtype)
    for s, k in enumerate(nodes):
        B[s, int(k)] = 1.0
    return B


def resample(m, src: tuple, dst: tuple) -> np.ndarray:
    """Bilinear resampling of a nodal model from grid src = (nx, nz, hx, hz)
    to grid dst over the same domain: the training model on a second grid,
    for data computed away from the inversion grid."""
    nx, nz, hx, hz = src
    mx, mz, gx, gz = dst
    M = np.asarray(m, dtype=np.float64).reshape(nz, nx)
    x = np.minimum(np.arange(mx) * gx / hx, nx - 1)
    z = np.minimum(np.arange(mz) * gz / hz, nz - 1)
    i = np.minimum(np.floor(x).astype(int), nx - 2)
    j = np.minimum(np.floor(z).astype(int), nz - 2)
    a = (x - i)[None, :]
    b = (z - j)[:, None]
    out = ((1 - a) * (1 - b) * M[j[:, None], i[None, :]] + a * (1 - b) * M[j[:, None], i[None, :] + 1]
           + (1 - a) * b * M[j[:, None] + 1, i[None, :]] + a * b * M[j[:, None] + 1, i[None, :] + 1])
    return np.ascontiguousarray(out.reshape(-1))
