"""Seeded synthetic inputs for ring-array sound-speed tomography.

This module produces *inputs* only: ring geometry, pixel grids, phantoms
(sound speed and absorption maps), frequency sets, start models and a
stand-in for measured transmission data.  It contains none of the
inversion's arithmetic (no ray tracing, no Green's functions on the grid,
no Born operators); both the FP64 oracle and the GPU library consume what
it returns.

Geometry conventions (shared by both implementations as an interface, not
as code):

* pixel (i, j) has its centre at ``(x0 + i*h, y0 + j*h)``; grids are stored
  row-major as ``[ny][nx]`` (row = j, column = i);
* ring element ``e`` sits at ``R*(cos(2*pi*e/m), sin(2*pi*e/m))`` around the
  origin, which is also the grid centre;
* the medium outside the grid is water at ``c_background`` with zero
  absorption.

The paper measures on the URMC in-vitro and in-vivo datasets (Results
section); those are not available, so the phantoms below stand in for them
with the same ring sizes, grid spacings, water speeds and frequency bands.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np
from scipy import ndimage

# 0.5 dB/(MHz cm) in Np/(m MHz): 0.5 dB/cm = 50 dB/m, 1 Np = 20/ln(10) dB.
DB_PER_MHZ_CM_TO_NP_PER_M_MHZ = 100.0 * math.log(10.0) / 20.0
TISSUE_ALPHA0 = 0.5 * DB_PER_MHZ_CM_TO_NP_PER_M_MHZ


@dataclass(frozen=True)
class Geometry:
    """Ring array plus pixel grid.  All lengths in metres, speeds in m/s."""

    nx: int
    ny: int
    h: float
    x0: float
    y0: float
    m: int
    ring_radius: float
    support_margin: float
    c_background: float

    @property
    def n_pixels(self) -> int:
        return self.nx * self.ny

    def pixel_centres(self) -> Tuple[np.ndarray, np.ndarray]:
        """Arrays X, Y of shape [ny][nx] with the pixel-centre coordinates."""
        xs = self.x0 + np.arange(self.nx, dtype=np.float64) * self.h
        ys = self.y0 + np.arange(self.ny, dtype=np.float64) * self.h
        return np.meshgrid(xs, ys, indexing="xy")

    def element_positions(self) -> np.ndarray:
        """[m][2] element positions, computed with the same libm calls as C."""
        out = np.empty((self.m, 2))
        for e in range(self.m):
            th = 2.0 * math.pi * e / self.m
            out[e, 0] = self.ring_radius * math.cos(th)
            out[e, 1] = self.ring_radius * math.sin(th)
        return out


@dataclass(frozen=True)
class TraceOpts:
    """Ray-fan options.  Zero means "use the default" for dtau/tau_max/j_min."""

    n_rays: int
    dtau: float = 0.0
    tau_max: float = 0.0
    j_min: float = 0.0


@dataclass(frozen=True)
class InvertOpts:
    recv_fraction: float = 0.75
    outlier_fraction: float = 0.01
    eps: float = 1e-3
    y_pow: float = 1.0


@dataclass
class Problem:
    """One reconstruction job: geometry, truth, start model, data, sets."""

    name: str
    geom: Geometry
    trace: TraceOpts
    inv: InvertOpts
    c_true: np.ndarray          # [ny][nx] m/s
    alpha0: np.ndarray          # [ny][nx] Np/(m MHz^y), a known model input
    c_start: np.ndarray         # [ny][nx] m/s
    freq_sets: List[np.ndarray]  # each an array of frequencies in Hz
    dtype: str                  # contraction dtype: f64 | f32 | bf16 | f16
    seed: int
    p_meas: List[np.ndarray] = field(default_factory=list)  # per set [nf][m][m] complex128

    @property
    def freqs(self) -> np.ndarray:
        return np.concatenate(self.freq_sets)


def centred_grid(n: int, h: float, m: int, ring_radius: float, c_bg: float,
                 support_margin: float | None = None) -> Geometry:
    x0 = -0.5 * (n - 1) * h
    if support_margin is None:
        support_margin = max(5e-3, 4.0 * h)
    return Geometry(nx=n, ny=n, h=h, x0=x0, y0=x0, m=m, ring_radius=ring_radius,
                    support_margin=support_margin, c_background=c_bg)


# ---------------------------------------------------------------------------
# phantoms
# ---------------------------------------------------------------------------

def _ellipse_mask(X, Y, cx, cy, a, b, ang):
    ca, sa = math.cos(ang), math.sin(ang)
    u = (X - cx) * ca + (Y - cy) * sa
    v = -(X - cx) * sa + (Y - cy) * ca
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def _disc_point(rng, radius):
    r = radius * math.sqrt(rng.uniform())
    t = 2.0 * math.pi * rng.uniform()
    return r * math.cos(t), r * math.sin(t)


def ellipse_phantom(geom: Geometry, seed: int, n_ellipses: int = 3,
                    c0: float = 1500.0, centre_radius: float = 18e-3):
    """Water plus seeded random ellipses (CPU-feasible case).

    Draw order per ellipse: semi-axis a, semi-axis b (both U[3,10] mm),
    angle U[0,pi), centre radius, centre angle, delta-c U[-30,30] m/s.
    Speeds add where ellipses overlap; 0.5 dB/(MHz cm) inside any ellipse.
    """
    rng = np.random.default_rng(seed)
    X, Y = geom.pixel_centres()
    c = np.full(X.shape, c0)
    inside_any = np.zeros(X.shape, bool)
    for _ in range(n_ellipses):
        a = rng.uniform(3e-3, 10e-3)
        b = rng.uniform(3e-3, 10e-3)
        ang = rng.uniform(0.0, math.pi)
        cx, cy = _disc_point(rng, centre_radius)
        dc = rng.uniform(-30.0, 30.0)
        msk = _ellipse_mask(X, Y, cx, cy, a, b, ang)
        c[msk] += dc
        inside_any |= msk
    alpha = np.where(inside_any, TISSUE_ALPHA0, 0.0)
    return c, alpha


def lens_medium(geom: Geometry, centre: Tuple[float, float], sigma: float, dc: float,
                c0: float = 1500.0, alpha0: float = 3.0):
    """Water with one Gaussian speed anomaly c0 + dc exp(-|x - centre|^2 /
    (2 sigma^2)) and a uniform absorption map.  A strong slow anomaly (dc of
    a few hundred m/s below c0, sigma a few pixels) a few millimetres in
    front of an element focuses that element's rays: its wavefront folds
    behind the lens (a caustic) and some points see several arrivals."""
    X, Y = geom.pixel_centres()
    c = c0 + dc * np.exp(-((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) / (2.0 * sigma ** 2))
    return c, np.full_like(c, alpha0)


def breast_phantom(geom: Geometry, seed: int, calcifications: bool = False,
                   support_radius: float | None = None):
    """Breast-like phantom: fat disc, fibroglandular blobs, inclusions, texture.

    * water 1500 m/s outside a disc of radius 0.8*R (or ``support_radius``);
    * fat 1470 m/s inside it;
    * 4-8 smoothed elliptical blobs, semi-axes U[10,30] mm, c U[1520,1560];
    * 5-15 inclusion discs, diameter U[2,8] mm, delta-c U[-40,40];
    * optionally 10-30 microcalcifications, diameter U[0.5,2] mm, +100 m/s;
    * Gaussian texture with 1 mm correlation length, sigma 5 m/s, inside;
    * 0.5 dB/(MHz cm) absorption inside the breast.
    """
    rng = np.random.default_rng(seed)
    X, Y = geom.pixel_centres()
    rb = 0.8 * geom.ring_radius if support_radius is None else support_radius
    rr = np.hypot(X, Y)
    inside = rr <= rb
    c = np.full(X.shape, 1500.0)
    c[inside] = 1470.0
    edge_px = max(1.0e-3 / geom.h, 0.5)
    n_blobs = int(rng.integers(4, 9))
    for _ in range(n_blobs):
        a = rng.uniform(10e-3, 30e-3) * rb / 88e-3
        b = rng.uniform(10e-3, 30e-3) * rb / 88e-3
        ang = rng.uniform(0.0, math.pi)
        cx, cy = _disc_point(rng, 0.55 * rb)
        cb = rng.uniform(1520.0, 1560.0)
        msk = _ellipse_mask(X, Y, cx, cy, a, b, ang).astype(np.float64)
        msk = ndimage.gaussian_filter(msk, edge_px) * inside
        c = c * (1.0 - msk) + cb * msk
    n_inc = int(rng.integers(5, 16))
    for _ in range(n_inc):
        d = rng.uniform(2e-3, 8e-3)
        cx, cy = _disc_point(rng, 0.7 * rb)
        dc = rng.uniform(-40.0, 40.0)
        c[(X - cx) ** 2 + (Y - cy) ** 2 <= (0.5 * d) ** 2] += dc
    if calcifications:
        n_cal = int(rng.integers(10, 31))
        for _ in range(n_cal):
            d = rng.uniform(0.5e-3, 2e-3)
            cx, cy = _disc_point(rng, 0.7 * rb)
            msk = (X - cx) ** 2 + (Y - cy) ** 2 <= (0.5 * d) ** 2
            if not msk.any():  # sub-pixel: mark the nearest pixel
                i = int(round((cx - geom.x0) / geom.h))
                j = int(round((cy - geom.y0) / geom.h))
                if 0 <= i < geom.nx and 0 <= j < geom.ny:
                    msk[j, i] = True
            c[msk] += 100.0
    noise = rng.standard_normal(X.shape)
    tex = ndimage.gaussian_filter(noise, 1.0e-3 / geom.h)
    sd = tex[inside].std() if inside.any() else 1.0
    c = c + np.where(inside, tex * (5.0 / sd), 0.0)
    alpha = np.where(inside, TISSUE_ALPHA0, 0.0)
    return c, alpha


def smoothed(c: np.ndarray, sigma_m: float, h: float, c_bg: float) -> np.ndarray:
    """Gaussian-smoothed copy of a speed map (stand-in for a ToF start model)."""
    return ndimage.gaussian_filter(c - c_bg, sigma_m / h) + c_bg


# ---------------------------------------------------------------------------
# measured-data stand-in
# ---------------------------------------------------------------------------

def straight_ray_data(geom: Geometry, c: np.ndarray, alpha: np.ndarray,
                      freqs: np.ndarray, y_pow: float = 1.0,
                      noise_rel: float = 0.0, seed: int = 0) -> np.ndarray:
    """Stand-in for measured transmission data, [nf][m][m] complex128.

    A deliberately *different* and simpler model than the inversion's:
    travel time and absorption are midpoint-rule line integrals of the
    nearest-pixel slowness and absorption along the straight chord e->r,
    the amplitude is the water-only 2-D far-field spreading
    sqrt(c_bg/(8 pi omega L)), with a +pi/4 phase.  Diagonal (e == r) is 0.
    """
    m = geom.m
    nf = len(freqs)
    out = np.zeros((nf, m, m), np.complex128)
    omega = 2.0 * math.pi * np.asarray(freqs, np.float64)
    fm = (np.asarray(freqs, np.float64) * 1e-6) ** y_pow
    rows = _chord_integrals(geom, c, alpha)
    for e in range(m):
        L, T, Bab = rows[e]
        with np.errstate(divide="ignore", invalid="ignore"):
            for k in range(nf):
                amp = np.sqrt(geom.c_background / (8.0 * math.pi * omega[k] * L))
                val = amp * np.exp(-Bab * fm[k]) * np.exp(1j * (omega[k] * T + 0.25 * math.pi))
                val[L == 0.0] = 0.0
                out[k, e, :] = val
    if noise_rel > 0.0:
        rng = np.random.default_rng(seed)
        rms = np.sqrt(np.mean(np.abs(out) ** 2, axis=(1, 2), keepdims=True))
        out = out + noise_rel * rms * (rng.standard_normal(out.shape)
                                       + 1j * rng.standard_normal(out.shape)) / math.sqrt(2.0)
    return out


def straight_ray_tof(geom: Geometry, c: np.ndarray) -> np.ndarray:
    """Stand-in for picked times of flight, [m][m] seconds: the straight-chord
    travel time of straight_ray_data (NaN for e == r)."""
    rows = _chord_integrals(geom, c, np.zeros_like(c))
    T = np.stack([r[1] for r in rows])
    T[np.arange(geom.m), np.arange(geom.m)] = np.nan
    return T


def _chord_integrals(geom: Geometry, c: np.ndarray, alpha: np.ndarray):
    """Per emitter: chord lengths, travel times and absorption integrals to
    every element (midpoint rule, nearest-pixel values, water outside)."""
    m = geom.m
    pos = geom.element_positions()
    s = 1.0 / c
    nsamp = int(math.ceil(2.0 * geom.ring_radius / (0.5 * geom.h)))
    t_mid = (np.arange(nsamp) + 0.5) / nsamp
    s_bg = 1.0 / geom.c_background

    def emitter_row(e):
        d = pos - pos[e]
        L = np.hypot(d[:, 0], d[:, 1])
        xs = pos[e, 0] + d[:, 0:1] * t_mid[None, :]
        ys = pos[e, 1] + d[:, 1:2] * t_mid[None, :]
        ii = np.rint((xs - geom.x0) / geom.h).astype(np.int64)
        jj = np.rint((ys - geom.y0) / geom.h).astype(np.int64)
        ok = (ii >= 0) & (ii < geom.nx) & (jj >= 0) & (jj < geom.ny)
        ic, jc = np.clip(ii, 0, geom.nx - 1), np.clip(jj, 0, geom.ny - 1)
        sv = np.where(ok, s[jc, ic], s_bg)
        av = np.where(ok, alpha[jc, ic], 0.0)
        return L, sv.sum(axis=1) * (L / nsamp), av.sum(axis=1) * (L / nsamp)

    # the chord integrals of different emitters are independent (threads:
    # NumPy releases the GIL in these array operations)
    workers = max(1, min(16, os.cpu_count() or 1)) if m >= 128 else 1
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(emitter_row, range(m)))
    return [emitter_row(e) for e in range(m)]


def random_tables(geom: Geometry, seed: int, t_scale: float | None = None,
                  uncovered_fraction: float = 0.02):
    """Seeded synthetic ray-to-grid tables, for testing the contractions alone.

    Returns T [m][N] float64 (NaN = uncovered), amp and att [m][N] float32
    and receiver tables T_rx [m][m], amp_rx, att_rx.  Values have the
    magnitudes of real tables (T up to 2R/c, amp ~ 5-50, att ~ 0-0.2).
    """
    rng = np.random.default_rng(seed)
    m, n = geom.m, geom.n_pixels
    if t_scale is None:
        t_scale = 2.0 * geom.ring_radius / geom.c_background
    T = rng.uniform(0.05, 1.0, (m, n)) * t_scale
    amp = rng.uniform(5.0, 50.0, (m, n)).astype(np.float32)
    att = rng.uniform(0.0, 0.2, (m, n)).astype(np.float32)
    T[rng.uniform(size=(m, n)) < uncovered_fraction] = np.nan
    Trx = rng.uniform(0.05, 1.0, (m, m)) * t_scale
    amp_rx = rng.uniform(5.0, 50.0, (m, m)).astype(np.float32)
    att_rx = rng.uniform(0.0, 0.2, (m, m)).astype(np.float32)
    return T, amp, att, Trx, amp_rx, att_rx


def random_delta(n: int, seed: int, scale: float = 1e-8) -> np.ndarray:
    """Seeded model perturbation (of squared slowness, s^2) for forward tests."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) * scale


def random_residual(nf: int, m: int, seed: int, scale: float = 1e-2) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal((nf, m, m)) + 1j * rng.standard_normal((nf, m, m)))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def _sets(freqs: np.ndarray, per_set: int) -> List[np.ndarray]:
    return [freqs[i:i + per_set].copy() for i in range(0, len(freqs), per_set)]


def data_for_sets(geom: Geometry, c: np.ndarray, alpha: np.ndarray,
                  freq_sets: List[np.ndarray]) -> List[np.ndarray]:
    """straight_ray_data for every set, the chord integrals taken once."""
    allf = np.concatenate([np.asarray(f, np.float64) for f in freq_sets])
    d = straight_ray_data(geom, c, alpha, allf)
    out, k = [], 0
    for f in freq_sets:
        out.append(np.ascontiguousarray(d[k:k + len(f)]))
        k += len(f)
    return out


def small_ring(seed: int = 1000, with_data: bool = True) -> Problem:
    """64-element ring, R = 30 mm, 128x128 grid at 0.5 mm, water plus three
    random ellipses; one set {200, 250} kHz; FP64; homogeneous start."""
    geom = centred_grid(128, 0.5e-3, 64, 30e-3, 1500.0)
    c, alpha = ellipse_phantom(geom, seed)
    freqs = np.array([200e3, 250e3])
    p = Problem("ring64_grid128", geom, TraceOpts(n_rays=360), InvertOpts(),
                c, alpha, np.full_like(c, 1500.0), [freqs], "f64", seed)
    if with_data:
        p.p_meas = data_for_sets(geom, c, alpha, p.freq_sets)
    return p


def small_ring_fullwave(seed: int = 1000, refine: int = 4) -> Problem:
    """The 64-element workload with full-wave data (Helmholtz FD on a grid
    `refine` times finer than the pixels) in place of the straight-ray
    stand-in: measured data from a wave model other than the inversion's."""
    from .fullwave import helmholtz_data
    p = small_ring(seed, with_data=False)
    p.p_meas = [helmholtz_data(p.geom, p.c_true, p.alpha0, f, y_pow=p.inv.y_pow, refine=refine)
                for f in p.freq_sets]
    p.name = p.name + "_fullwave"
    return p


def breast_ring256(seed: int = 1001, with_data: bool = True, dtype: str = "f32") -> Problem:
    """256-element ring, R = 110 mm, 480x480 grid at 0.5 mm, breast phantom;
    24 frequencies 0.3-1.25 MHz in 8 sets of 3; start = truth smoothed 4 mm."""
    geom = centred_grid(480, 0.5e-3, 256, 110e-3, 1500.0)
    c, alpha = breast_phantom(geom, seed)
    freqs = np.linspace(0.3e6, 1.25e6, 24)
    p = Problem("ring256_grid480", geom, TraceOpts(n_rays=720), InvertOpts(),
                c, alpha, smoothed(c, 4e-3, geom.h, 1500.0), _sets(freqs, 3), dtype, seed)
    if with_data:
        p.p_meas = data_for_sets(geom, c, alpha, p.freq_sets)
    return p


def breast_ring1024(seed: int = 1003, with_data: bool = True, dtype: str = "bf16") -> Problem:
    """1024-element ring, R = 110 mm, 1100x1100 grid at 0.2 mm, breast phantom
    with microcalcifications; 48 frequencies 0.3-2.0 MHz in 12 sets of 4."""
    geom = centred_grid(1100, 0.2e-3, 1024, 110e-3, 1500.0)
    c, alpha = breast_phantom(geom, seed, calcifications=True)
    freqs = np.linspace(0.3e6, 2.0e6, 48)
    p = Problem("ring1024_grid1100", geom, TraceOpts(n_rays=1440), InvertOpts(),
                c, alpha, smoothed(c, 4e-3, geom.h, 1500.0), _sets(freqs, 4), dtype, seed)
    if with_data:
        p.p_meas = data_for_sets(geom, c, alpha, p.freq_sets)
    return p


def custom(n: int, h: float, m: int, ring_radius: float, n_rays: int,
           freq_sets: List[List[float]], seed: int = 7, kind: str = "ellipses",
           dtype: str = "f64", with_data: bool = True, ny: int | None = None) -> Problem:
    """A small problem of arbitrary shape (parity tests: ragged grids etc.)."""
    geom = centred_grid(n, h, m, ring_radius, 1500.0)
    if ny is not None and ny != n:
        geom = dataclasses.replace(geom, ny=ny, y0=-0.5 * (ny - 1) * h)
    if kind == "ellipses":
        c, alpha = ellipse_phantom(geom, seed, centre_radius=0.6 * ring_radius)
        start = np.full_like(c, 1500.0)
    elif kind == "breast":
        c, alpha = breast_phantom(geom, seed, support_radius=0.8 * min(ring_radius, 0.5 * n * h))
        start = smoothed(c, 4e-3, h, 1500.0)
    elif kind == "water":
        c, alpha = np.full((geom.ny, geom.nx), 1500.0), np.zeros((geom.ny, geom.nx))
        start = c.copy()
    else:
        raise ValueError(kind)
    sets = [np.asarray(f, np.float64) for f in freq_sets]
    p = Problem(f"custom_{kind}_{n}_{m}", geom, TraceOpts(n_rays=n_rays), InvertOpts(),
                c, alpha, start, sets, dtype, seed)
    if with_data:
        p.p_meas = data_for_sets(geom, c, alpha, p.freq_sets)
    return p


def serving_stream(n_jobs: int = 200, rate: float = 0.5, seed: int = 42,
                   mix=(5, 4, 1)):
    """Poisson job stream mixing the three sizes; returns a list of dicts with
    arrival time, size class and per-job phantom seed and ring radius."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    p = np.asarray(mix, np.float64) / float(sum(mix))
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        cls = int(rng.choice(3, p=p))
        radius = rng.uniform(80e-3, 120e-3)
        jobs.append({"job": j, "arrival_s": t, "size_class": cls,
                     "seed": 2000 + j, "ring_radius": radius})
    return jobs


SERVING_CLASSES = ("ring64_grid128", "ring256_grid480", "ring1024_grid1100")


def serving_job(size_class: int, seed: int, ring_radius: float, with_data: bool = True,
                dtype: str = "f32") -> Problem:
    """One job of the serving stream: the grid, ring size and frequency sets
    of the 64-, 256- or 1024-element workloads, with the job's own ring
    radius and seeded phantom (support scaled to min(R, half grid))."""
    if size_class == 0:
        n, h, m, n_rays = 128, 0.5e-3, 64, 360
        sets = [np.array([200e3, 250e3])]
    elif size_class == 1:
        n, h, m, n_rays = 480, 0.5e-3, 256, 720
        sets = _sets(np.linspace(0.3e6, 1.25e6, 24), 3)
    elif size_class == 2:
        n, h, m, n_rays = 1100, 0.2e-3, 1024, 1440
        sets = _sets(np.linspace(0.3e6, 2.0e6, 48), 4)
    else:
        raise ValueError(size_class)
    geom = centred_grid(n, h, m, ring_radius, 1500.0)
    support = min(ring_radius, 0.5 * n * h)
    if size_class == 0:
        c, alpha = ellipse_phantom(geom, seed, centre_radius=0.6 * support)
        start = np.full_like(c, 1500.0)
    else:
        c, alpha = breast_phantom(geom, seed, support_radius=0.8 * support, calcifications=size_class == 2)
        start = smoothed(c, 4e-3, h, 1500.0)
    p = Problem(f"{SERVING_CLASSES[size_class]}_job{seed}", geom, TraceOpts(n_rays=n_rays), InvertOpts(),
                c, alpha, start, sets, dtype, seed)
    if with_data:
        p.p_meas = data_for_sets(geom, c, alpha, p.freq_sets)
    return p


def resolve_trace_opts(geom: Geometry, c: np.ndarray, n_rays: int,
                       headroom: float = 1.1) -> TraceOpts:
    """Fix the ray step and length for a job from its start model.

    dtau = h / (2 c_hi) and tau_max = 2.5 R / c_lo, where c_hi and c_lo are
    the largest and smallest speeds of the start model and the water,
    widened by ``headroom`` so later sets of the sweep keep the same step.
    j_min = h / 4 bounds the ray-tube width at the source."""
    c_hi = max(float(np.max(c)), geom.c_background) * headroom
    c_lo = min(float(np.min(c)), geom.c_background) / headroom
    return TraceOpts(n_rays=n_rays, dtau=geom.h / (2.0 * c_hi),
                     tau_max=2.5 * geom.ring_radius / c_lo, j_min=0.25 * geom.h)
