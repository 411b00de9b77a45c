"""Seeded synthetic inputs for the preconditioned FWI gradient.

This module builds *inputs only*: velocity models, acquisition geometry,
source wavelets and perturbation directions.  It contains none of the
method's arithmetic (no propagation, misfit, adjoint, imaging or Hessian
work), so the FP64 oracle and the HIP path can both be fed from it.

The paper's own workload is the 2D Marmousi model with 80 shots and
full-aperture receivers (section 2.1) and a Gaussian-smoothed Marmousi start
model (section 3.1).  Marmousi is not available here; a seeded layered model
with the same velocity range as the paper's start model (1.5 to 4.5 km/s,
section 2.1) stands in for it.

Conventions used throughout the package:

* model grid ``[nz][nx]``, row-major, x contiguous, ``dz == dx``;
* shot/receiver positions are model-grid cell indices ``(iz, ix)``;
* receivers of all shots are stored as a CSR list: shot ``s`` owns
  ``rec_iz[rec_ptr[s]:rec_ptr[s+1]]``;
* each shot has its own record length ``nt[s] <= nt_max``; traces are
  stored ``[ntrace][nt_max]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter


# --------------------------------------------------------------------------
# plain containers
# --------------------------------------------------------------------------
@dataclass
class Grid:
    nz: int
    nx: int
    dx: float          # metres, dz == dx
    dt: float          # seconds
    nt_max: int
    nsponge: int       # absorbing-sponge width N (cells) padded on all 4 sides
    v_ref: float       # sponge reference velocity (m/s), not differentiated
    free_surface: bool = False   # pressure-free top instead of the top sponge

    @property
    def padded(self):
        return (self.nz + 2 * self.nsponge, self.nx + 2 * self.nsponge)


@dataclass
class Geometry:
    src_iz: np.ndarray          # int32 [nshot]
    src_ix: np.ndarray          # int32 [nshot]
    rec_ptr: np.ndarray         # int32 [nshot+1]
    rec_iz: np.ndarray          # int32 [ntrace]
    rec_ix: np.ndarray          # int32 [ntrace]
    nt: np.ndarray              # int32 [nshot]

    @property
    def nshot(self) -> int:
        return int(self.src_iz.shape[0])

    @property
    def ntrace(self) -> int:
        return int(self.rec_ptr[-1])

    def shot(self, s: int):
        """(src_iz, src_ix, rec_iz[], rec_ix[], nt) of shot s."""
        a, b = int(self.rec_ptr[s]), int(self.rec_ptr[s + 1])
        return (int(self.src_iz[s]), int(self.src_ix[s]),
                self.rec_iz[a:b], self.rec_ix[a:b], int(self.nt[s]))

    def subset(self, shots) -> "Geometry":
        shots = [int(s) for s in shots]
        iz, ix, ptr = [], [], [0]
        for s in shots:
            a, b = int(self.rec_ptr[s]), int(self.rec_ptr[s + 1])
            iz.append(self.rec_iz[a:b]); ix.append(self.rec_ix[a:b])
            ptr.append(ptr[-1] + (b - a))
        return Geometry(
            src_iz=self.src_iz[shots].astype(np.int32).copy(),
            src_ix=self.src_ix[shots].astype(np.int32).copy(),
            rec_ptr=np.asarray(ptr, np.int32),
            rec_iz=np.concatenate(iz).astype(np.int32),
            rec_ix=np.concatenate(ix).astype(np.int32),
            nt=self.nt[shots].astype(np.int32).copy())

    def with_nt(self, nt: int) -> "Geometry":
        """Same geometry with every record truncated to ``min(nt_s, nt)``."""
        g = Geometry(self.src_iz.copy(), self.src_ix.copy(), self.rec_ptr.copy(),
                     self.rec_iz.copy(), self.rec_ix.copy(),
                     np.minimum(self.nt, nt).astype(np.int32))
        return g


@dataclass
class Workload:
    name: str
    grid: Grid
    geom: Geometry
    v_true: np.ndarray          # float32 [nz][nx]
    v_start: np.ndarray         # float32 [nz][nx]
    wavelet: np.ndarray         # float32 [nt_max] (shared by all shots)
    f_peak: float
    hmax: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# wavelet and models
# --------------------------------------------------------------------------
def ricker(f_peak: float, dt: float, nt: int, t0: Optional[float] = None,
           amplitude: float = 1.0) -> np.ndarray:
    """Ricker wavelet sampled at t = n*dt, delay t0 = 1.5/f_peak by default."""
    if t0 is None:
        t0 = 1.5 / f_peak
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (np.pi * f_peak * t) ** 2
    return amplitude * (1.0 - 2.0 * a) * np.exp(-a)


def gaussian_anomaly(nz, nx, v0=2000.0, rel_amp=0.1, sigma=8.0, iz0=None, ix0=None):
    """v0 * (1 + rel_amp * exp(-r^2 / (2 sigma^2))), r in cells."""
    iz0 = nz // 2 if iz0 is None else iz0
    ix0 = nx // 2 if ix0 is None else ix0
    z = np.arange(nz)[:, None] - iz0
    x = np.arange(nx)[None, :] - ix0
    return (v0 * (1.0 + rel_amp * np.exp(-(z * z + x * x) / (2.0 * sigma * sigma)))).astype(np.float32)


def layered_model(nz, nx, dx, seed=1406, n_if=12, vmin=1500.0, vmax=4500.0, max_dip_deg=12.0):
    """Seeded layered model with dipping interfaces, defined in physical units so that
    the same seed gives the same geology at any resolution."""
    rng = np.random.default_rng(seed)
    Lx, Lz = nx * dx, nz * dx
    zi = np.sort(rng.uniform(0.04, 0.96, n_if)) * Lz
    dip = np.deg2rad(rng.uniform(-max_dip_deg, max_dip_deg, n_if))
    vk = vmin + (vmax - vmin) * np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0.0, 1.0, n_if - 1)]))
    x = np.arange(nx) * dx
    z = np.arange(nz) * dx
    layer = np.zeros((nz, nx), np.int64)
    for i in range(n_if):
        zif = zi[i] + np.tan(dip[i]) * (x - 0.5 * Lx)
        layer += (z[:, None] > zif[None, :])
    return vk[layer].astype(np.float32)


def smooth(v, sigma_cells):
    return gaussian_filter(v.astype(np.float64), sigma=sigma_cells, mode="nearest").astype(np.float32)


def surface_geometry(src_ix, rec_ix_per_shot: List[np.ndarray], src_iz, rec_iz, nt_per_shot) -> Geometry:
    nshot = len(src_ix)
    ptr = np.zeros(nshot + 1, np.int32)
    for s, r in enumerate(rec_ix_per_shot):
        ptr[s + 1] = ptr[s] + len(r)
    rix = np.concatenate(rec_ix_per_shot).astype(np.int32)
    return Geometry(
        src_iz=np.full(nshot, src_iz, np.int32),
        src_ix=np.asarray(src_ix, np.int32),
        rec_ptr=ptr,
        rec_iz=np.full(rix.shape[0], rec_iz, np.int32),
        rec_ix=rix,
        nt=np.asarray(nt_per_shot, np.int32) * np.ones(nshot, np.int32))


# --------------------------------------------------------------------------
# the five workloads (names describe the workload)
# --------------------------------------------------------------------------
def anomaly_200x100() -> Workload:
    """One shot over a +10 % Gaussian anomaly: 200x100 cells, dx=10 m, 20-cell sponge,
    Ricker 10 Hz at depth 2 cells, 100 surface receivers, dt=1 ms, nt=1000."""
    nz, nx, dx = 100, 200, 10.0
    v_true = gaussian_anomaly(nz, nx, 2000.0, 0.1, 8.0, iz0=50, ix0=100)
    v_start = np.full((nz, nx), 2000.0, np.float32)
    nt = 1000
    grid = Grid(nz, nx, dx, 1e-3, nt, 20, float(v_true.max()))
    geom = surface_geometry([100], [np.arange(0, 200, 2)], 2, 2, nt)
    return Workload("anomaly_200x100_1shot_nt1000", grid, geom, v_true, v_start,
                    ricker(10.0, 1e-3, nt).astype(np.float32), 10.0)


def layered_1024x384(nshot=64, nt=4000) -> Workload:
    """Seeded 12-interface layered model, 1024x384 cells, dx=12.5 m, 32-cell sponge;
    64 shots at depth 2 (ix = 16k+8), 512 fixed-spread receivers (ix = 2k),
    Ricker 8 Hz, dt = 1 ms, nt = 4000.  Start model: Gaussian smoothing, 20 cells."""
    nz, nx, dx = 384, 1024, 12.5
    v_true = layered_model(nz, nx, dx, seed=1406)
    v_start = smooth(v_true, 20.0)
    grid = Grid(nz, nx, dx, 1e-3, nt, 32, float(v_true.max()))
    src = 16 * np.arange(64) + 8
    src = src[:nshot]
    geom = surface_geometry(src, [np.arange(0, 1024, 2)] * len(src), 2, 2, nt)
    return Workload(f"layered_1024x384_{nshot}shots_nt{nt}", grid, geom, v_true, v_start,
                    ricker(8.0, 1e-3, nt).astype(np.float32), 8.0)


def ragged_1024x384(nshot=256) -> Workload:
    """256 shots of uneven aperture (128..1024 contiguous receivers centred on the
    shot) and uneven record length (nt 2000..6000) on the 1024x384 layered model."""
    base = layered_1024x384(nshot=1)
    rng = np.random.default_rng(1864)
    nx = base.grid.nx
    ix_s = rng.integers(0, nx, nshot)
    nrec = rng.integers(128, 1025, nshot)
    nt_s = rng.integers(2000, 6001, nshot)
    recs = []
    for s in range(nshot):
        n = int(nrec[s])
        a = int(ix_s[s]) - n // 2
        a = min(max(a, 0), nx - n)
        recs.append(np.arange(a, a + n))
    nt_max = int(nt_s.max())
    geom = surface_geometry(ix_s, recs, 2, 2, 1)
    geom.nt = nt_s.astype(np.int32)
    grid = Grid(base.grid.nz, nx, base.grid.dx, base.grid.dt, nt_max, base.grid.nsponge, base.grid.v_ref)
    return Workload(f"ragged_1024x384_{nshot}shots", grid, geom, base.v_true, base.v_start,
                    ricker(8.0, 1e-3, nt_max).astype(np.float32), 8.0)


def autograd_1024x384() -> Workload:
    """Shots 0, 2, ..., 62 of the 1024x384 layered workload (32 shots, nt = 4000)."""
    w = layered_1024x384()
    w.geom = w.geom.subset(range(0, 64, 2))
    w.name = "layered_1024x384_32shots_nt4000_autograd"
    return w


def offset_2048x768(nshot=32, nt=8000) -> Workload:
    """Same layered geology at dx = 6.25 m: 2048x768 cells, 64-cell sponge,
    32 shots at depth 4 (ix = 64k+32), 1024 receivers (ix = 2k), Ricker 15 Hz,
    dt = 0.5 ms, nt = 8000, horizontal subsurface offsets |h| <= 16 cells."""
    nz, nx, dx = 768, 2048, 6.25
    v_true = layered_model(nz, nx, dx, seed=1406)
    v_start = smooth(v_true, 40.0)
    grid = Grid(nz, nx, dx, 5e-4, nt, 64, float(v_true.max()))
    src = (64 * np.arange(32) + 32)[:nshot]
    geom = surface_geometry(src, [np.arange(0, 2048, 2)] * len(src), 4, 4, nt)
    return Workload(f"layered_2048x768_{nshot}shots_nt{nt}_offset16", grid, geom, v_true, v_start,
                    ricker(15.0, 5e-4, nt).astype(np.float32), 15.0, hmax=16)


def tiny_24x16(nt=400) -> Workload:
    """Small brute-force grid: 24x16 cells, dx=10 m, 8-cell sponge, dt=1 ms,
    v = 2000 (1 + 0.1 Gaussian(sigma 3 cells)), 2 shots at depth 1 (ix 3, 20),
    6 receivers at depth 1 (ix 2, 6, ..., 22), Ricker 10 Hz."""
    nz, nx, dx = 16, 24, 10.0
    v_true = gaussian_anomaly(nz, nx, 2000.0, 0.1, 3.0, iz0=8, ix0=12)
    v_start = np.full((nz, nx), 2000.0, np.float32)
    grid = Grid(nz, nx, dx, 1e-3, nt, 8, float(v_true.max()))
    geom = surface_geometry([3, 20], [np.arange(2, 24, 4)] * 2, 1, 1, nt)
    return Workload(f"tiny_24x16_nt{nt}", grid, geom, v_true, v_start,
                    ricker(10.0, 1e-3, nt).astype(np.float32), 10.0, hmax=2)


def layered_256x96(nshot=16, nt=1500) -> Workload:
    """The layered geology at dx = 50 m for iterative inversions: 256x96 cells
    (12.8 x 4.8 km), 16-cell sponge, 16 shots at depth 1 (ix = 16k+8), 128
    receivers (ix = 2k), Ricker 3 Hz, dt = 4 ms, nt = 1500 (6 s).  Start model:
    Gaussian smoothing, 5 cells (the 250 m of the 1024x384 workload)."""
    nz, nx, dx = 96, 256, 50.0
    v_true = layered_model(nz, nx, dx, seed=1406)
    v_start = smooth(v_true, 5.0)
    grid = Grid(nz, nx, dx, 4e-3, nt, 16, float(v_true.max()))
    src = (16 * np.arange(16) + 8)[:nshot]
    geom = surface_geometry(src, [np.arange(0, 256, 2)] * len(src), 1, 1, nt)
    return Workload(f"layered_256x96_{nshot}shots_nt{nt}", grid, geom, v_true, v_start,
                    ricker(3.0, 4e-3, nt).astype(np.float32), 3.0, hmax=8)


WORKLOADS = {
    "anomaly_200x100": anomaly_200x100,
    "layered_1024x384": layered_1024x384,
    "ragged_1024x384": ragged_1024x384,
    "autograd_1024x384": autograd_1024x384,
    "offset_2048x768": offset_2048x768,
    "layered_256x96": layered_256x96,
}


# --------------------------------------------------------------------------
# perturbation directions for directional-derivative checks
# --------------------------------------------------------------------------
def bump_direction(nz, nx, sigma=16.0):
    z = np.arange(nz)[:, None] - nz / 2.0
    x = np.arange(nx)[None, :] - nx / 2.0
    return np.exp(-(z * z + x * x) / (2 * sigma * sigma))


def noise_direction(nz, nx, seed=2014, sigma=8.0, taper=12):
    rng = np.random.default_rng(seed)
    d = gaussian_filter(rng.standard_normal((nz, nx)), sigma=sigma, mode="nearest")
    m = np.zeros((nz, nx))
    m[taper:nz - taper, taper:nx - taper] = 1.0
    return d * m


def random_traces(geom: Geometry, nt_max: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded band-limited stand-in for recorded data, zero past each shot's nt."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((geom.ntrace, nt_max))
    d = gaussian_filter(d, sigma=(0, 6.0), mode="nearest") * scale
    for s in range(geom.nshot):
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        d[a:b, int(geom.nt[s]):] = 0.0
    return d.astype(np.float32)
