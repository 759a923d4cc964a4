"""Seeded synthetic inputs shaped like the paper's workloads (Section IV-B).

This module only draws inputs: grids, velocity models, off-grid source and
receiver coordinates and source wavelets. It holds none of the propagator's
arithmetic, so both the FP64 oracle and the HIP path can consume the same
arrays. Everything is drawn from ``numpy.random.Generator(PCG64(seed))``.

The paper benchmarks unspecified synthetic 512^3 velocity models with one
seismic source wavelet, zero initial conditions and absorbing layers
(Section IV-B); no public dataset is involved. The recipes below follow the
workload table of the design notes (two-layer and Gaussian-filtered models,
Ricker wavelets, sources uniform in the non-sponge interior, receivers on an
off-grid line parallel to x).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ACOUSTIC, TTI, ELASTIC = 0, 1, 2


@dataclasses.dataclass
class Shot:
    """One propagation problem: a model on a grid plus sparse operators.

    Arrays are C-order ``[nx][ny][nz]`` (z fastest). Coordinates are in metres,
    ``src_xyz``/``rec_xyz`` are ``[npts][3]`` float64, ``src_wav`` is
    ``[nt][nsrc]`` float64 (the value injected at ``t_n = n*dt``).
    """

    shape: tuple
    spacing: tuple
    origin: tuple
    space_order: int
    nbl: int
    dt: float
    nt: int
    vp: np.ndarray
    src_xyz: np.ndarray
    src_wav: np.ndarray
    rec_xyz: np.ndarray
    physics: int = ACOUSTIC
    # TTI parameters
    epsilon: Optional[np.ndarray] = None
    delta: Optional[np.ndarray] = None
    theta: Optional[np.ndarray] = None
    phi: Optional[np.ndarray] = None
    # elastic parameters
    vs: Optional[np.ndarray] = None
    rho: Optional[np.ndarray] = None
    seed: int = 0
    name: str = ""

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))

    def extent(self):
        return [(n - 1) * h for n, h in zip(self.shape, self.spacing)]


def ricker(f0: float, nt: int, dt: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet sampled at t_n = n*dt, unit amplitude, delay t0 = 1/f0."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _interior_uniform(rng, shape, spacing, origin, nbl, npts):
    """Uniform off-grid points strictly inside the non-sponge interior."""
    lo = np.array([o + nbl * h for o, h in zip(origin, spacing)])
    hi = np.array([o + (n - 1 - nbl) * h for o, n, h in zip(origin, shape, spacing)])
    return lo + (hi - lo) * rng.random((npts, 3))


def _receiver_line_x(rng, shape, spacing, origin, nbl, nrec, jitter=0.25):
    """nrec receivers on a line parallel to x at a random off-grid (y0, z0).

    x_i = (i + 0.5 + j) * L / nrec over the full x range, with one random
    sub-cell offset j in [0, jitter) for the whole line.
    """
    n = shape
    h = spacing
    lo_y = origin[1] + nbl * h[1]
    hi_y = origin[1] + (n[1] - 1 - nbl) * h[1]
    lo_z = origin[2] + nbl * h[2]
    hi_z = origin[2] + (n[2] - 1 - nbl) * h[2]
    y0 = lo_y + (hi_y - lo_y) * rng.random()
    z0 = lo_z + (hi_z - lo_z) * rng.random()
    j = jitter * rng.random()
    L = (n[0] - 1) * h[0]
    x = origin[0] + (np.arange(nrec) + 0.5 + j) * L / nrec
    x = np.minimum(x, origin[0] + L)
    rec = np.empty((nrec, 3))
    rec[:, 0] = x
    rec[:, 1] = y0
    rec[:, 2] = z0
    return rec


def _receiver_line_interior(rng, shape, spacing, origin, nbl, nrec):
    """nrec receivers evenly over the interior x-range, random sub-cell offset."""
    h = spacing
    lo = origin[0] + nbl * h[0]
    hi = origin[0] + (shape[0] - 1 - nbl) * h[0]
    lo_y = origin[1] + nbl * h[1]
    hi_y = origin[1] + (shape[1] - 1 - nbl) * h[1]
    lo_z = origin[2] + nbl * h[2]
    hi_z = origin[2] + (shape[2] - 1 - nbl) * h[2]
    y0 = lo_y + (hi_y - lo_y) * rng.random()
    z0 = lo_z + (hi_z - lo_z) * rng.random()
    off = rng.random() * h[0]
    x = lo + off + np.arange(nrec) * (hi - lo - h[0]) / max(nrec - 1, 1)
    rec = np.empty((nrec, 3))
    rec[:, 0] = x
    rec[:, 1] = y0
    rec[:, 2] = z0
    return rec


def cfl_dt(vmax: float, h: float, cfl: float = 0.4) -> float:
    return cfl * h / vmax


def two_layer_vp(rng, shape, v_top=1500.0, v_bot=4500.0, frac=(0.25, 0.75)):
    """Two-layer velocity: v_top above a random depth index, v_bot below."""
    nz = shape[2]
    zint = int(round((frac[0] + (frac[1] - frac[0]) * rng.random()) * (nz - 1)))
    vp = np.empty(shape, dtype=np.float64)
    vp[..., :zint] = v_top
    vp[..., zint:] = v_bot
    return vp, zint


def smooth_field(rng, shape, lo, hi, sigma=8.0):
    """Gaussian-filtered N(0,1) noise (reflective edges), min-max mapped."""
    from scipy.ndimage import gaussian_filter

    g = gaussian_filter(rng.standard_normal(shape), sigma=sigma, mode="reflect")
    g = (g - g.min()) / max(g.max() - g.min(), 1e-300)
    return lo + (hi - lo) * g


def acoustic_small(seed: int = 10249, n: int = 64, so: int = 4, nt: int = 100,
                   nbl: int = 10, h: float = 10.0, vp0: float = 1500.0,
                   f0: float = 10.0, nrec: int = 32, nsrc: int = 1) -> Shot:
    """Isotropic acoustic parity case: n^3, constant vp, one off-grid Ricker
    source in the non-sponge interior and a line of receivers along x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    dt = cfl_dt(vp0, h)
    vp = np.full(shape, vp0, dtype=np.float64)
    src = _interior_uniform(rng, shape, spacing, origin, nbl, nsrc)
    wav = np.stack([ricker(f0, nt, dt) for _ in range(nsrc)], axis=1)
    rec = _receiver_line_interior(rng, shape, spacing, origin, nbl, nrec)
    return Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                seed=seed, name=f"acoustic {n}^3 SO{so} nt={nt}")


def acoustic_two_layer(seed: int = 10250, n=512, so: int = 8, nt: int = 1000,
                       nbl: int = 40, h: float = 10.0, nsrc: int = 8,
                       nrec: Optional[int] = None, fband=(8.0, 15.0),
                       v_top=1500.0, v_bot=4500.0) -> Shot:
    """Two-layer acoustic roofline case (default 512^3 SO8, 1000 steps, 8
    sources with f ~ U[8, 15] Hz, 512 receivers on an x-line)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    vp, _ = two_layer_vp(rng, shape, v_top, v_bot)
    dt = cfl_dt(max(v_top, v_bot), h)
    src = _interior_uniform(rng, shape, spacing, origin, nbl, nsrc)
    f = fband[0] + (fband[1] - fband[0]) * rng.random(nsrc)
    wav = np.stack([ricker(fi, nt, dt) for fi in f], axis=1)
    if nrec is None:
        nrec = shape[0]
    rec = _receiver_line_x(rng, shape, spacing, origin, nbl, nrec)
    return Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                seed=seed, name=f"acoustic two-layer {shape[0]}^3 SO{so} nt={nt}")


def acoustic_source_density(nsrc: int, layout: str = "volume", seed: int = 10254, n=512,
                            so: int = 8, nt: int = 1000, nbl: int = 40, h: float = 10.0):
    """The two-layer case with many sources (Section IV-E's stress test):
    `layout` "volume" draws them uniformly in the interior, "plane" on a
    horizontal plane at a random off-grid depth (sources on a plane of the
    blocked y-z tiles). Wavelets are Ricker with f ~ U[8, 15] Hz."""
    shot = acoustic_two_layer(seed=seed, n=n, so=so, nt=nt, nbl=nbl, h=h, nsrc=1)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    src = _interior_uniform(rng, shot.shape, shot.spacing, shot.origin, nbl, nsrc)
    if layout == "plane":
        src[:, 2] = src[0, 2]
    elif layout != "volume":
        raise ValueError(f"layout {layout!r}")
    f = 8.0 + 7.0 * rng.random(nsrc)
    shot.src_xyz = src
    shot.src_wav = np.stack([ricker(fi, nt, shot.dt) for fi in f], axis=1)
    shot.name = f"acoustic two-layer {shot.shape[0]}^3 SO{so} nt={nt}, {nsrc} sources ({layout})"
    return shot


def acoustic_scaled(seed: int, n: int, so: int, nt: int, nbl: int, nsrc: int = 1,
                    nrec: int = 16, layered: bool = True, h: float = 10.0) -> Shot:
    """Small two-layer (or constant) acoustic case for tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    if layered:
        vp, _ = two_layer_vp(rng, shape)
    else:
        vp = np.full(shape, 1500.0)
    dt = cfl_dt(float(vp.max()), h)
    src = _interior_uniform(rng, shape, spacing, origin, nbl, nsrc)
    f = 8.0 + 7.0 * rng.random(nsrc)
    wav = np.stack([ricker(fi, nt, dt) for fi in f], axis=1)
    rec = _receiver_line_x(rng, shape, spacing, origin, nbl, nrec)
    return Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                seed=seed, name=f"acoustic {shape} SO{so} nt={nt}")


def tti_smooth(seed: int = 10251, n: int = 256, so: int = 8, nt: int = 800,
               nbl: int = 20, h: float = 20.0, nsrc: int = 4, nrec: int = 256,
               sigma: float = 8.0, f0: float = 10.0) -> Shot:
    """TTI case: smooth random vp, epsilon, delta, theta, phi (Section III-B)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    sub = [np.random.Generator(np.random.PCG64(seed * 16 + k)) for k in range(5)]
    vp = smooth_field(sub[0], shape, 1500.0, 4500.0, sigma)
    eps = smooth_field(sub[1], shape, 0.0, 0.3, sigma)
    dlt = smooth_field(sub[2], shape, 0.0, 0.15, sigma)
    dlt = np.minimum(dlt, eps)
    th = smooth_field(sub[3], shape, -math.pi / 4, math.pi / 4, sigma)
    ph = smooth_field(sub[4], shape, -math.pi / 4, math.pi / 4, sigma)
    veff = float((vp * np.sqrt(1.0 + 2.0 * eps)).max())
    dt = cfl_dt(veff, h)
    src = _interior_uniform(rng, shape, spacing, origin, nbl, nsrc)
    wav = np.stack([ricker(f0, nt, dt) for _ in range(nsrc)], axis=1)
    rec = _receiver_line_x(rng, shape, spacing, origin, nbl, nrec)
    return Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                physics=TTI, epsilon=eps, delta=dlt, theta=th, phi=ph,
                seed=seed, name=f"tti {shape[0]}^3 SO{so} nt={nt}")


def elastic_smooth(seed: int = 10252, n: int = 256, so: int = 8, nt: int = 600,
                   nbl: int = 20, h: float = 10.0, nrec: int = 256,
                   sigma: float = 8.0, f0: float = 10.0) -> Shot:
    """Elastic case: smooth vp in [2000, 4000], vs = vp/1.8, rho in
    [1800, 2600] (Section III-C)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    sub = [np.random.Generator(np.random.PCG64(seed * 16 + k)) for k in range(2)]
    vp = smooth_field(sub[0], shape, 2000.0, 4000.0, sigma)
    vs = vp / 1.8
    rho = smooth_field(sub[1], shape, 1800.0, 2600.0, sigma)
    dt = cfl_dt(float(vp.max()), h)
    src = _interior_uniform(rng, shape, spacing, origin, nbl, 1)
    wav = ricker(f0, nt, dt)[:, None]
    rec = _receiver_line_x(rng, shape, spacing, origin, nbl, nrec)
    return Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                physics=ELASTIC, vs=vs, rho=rho,
                seed=seed, name=f"elastic {shape[0]}^3 SO{so} nt={nt}")


def serving_request(rng, sizes=(128, 192, 256, 384), nt_range=(500, 1500),
                    so: int = 8, nbl: int = 20, h: float = 10.0):
    """One serving request: a two-layer model, one Ricker source near the top
    (z = nbl + 2 cells), a receiver line of N receivers at the same depth, and
    a 'true' model (+5% vp Gaussian blob of radius 8 cells) for observed data."""
    n = int(rng.choice(sizes))
    nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
    shape = (n, n, n)
    spacing = (h, h, h)
    origin = (0.0, 0.0, 0.0)
    vp, _ = two_layer_vp(rng, shape)
    dt = cfl_dt(4500.0, h)
    f0 = 8.0 + 7.0 * rng.random()
    zs = (nbl + 2) * h
    lo = nbl * h
    hi = (n - 1 - nbl) * h
    src = np.array([[lo + (hi - lo) * rng.random(), lo + (hi - lo) * rng.random(), zs]])
    wav = ricker(f0, nt, dt)[:, None]
    rec = np.empty((n, 3))
    rec[:, 0] = (np.arange(n) + 0.5) * (n - 1) * h / n
    rec[:, 1] = src[0, 1]
    rec[:, 2] = zs
    c = lo / h + (hi - lo) / h * rng.random(3)
    ii = np.arange(n, dtype=np.float64)
    r2 = ((ii[:, None, None] - c[0]) ** 2 + (ii[None, :, None] - c[1]) ** 2
          + (ii[None, None, :] - c[2]) ** 2)
    vp_true = vp * (1.0 + 0.05 * np.exp(-r2 / (2 * 8.0 ** 2)))
    shot = Shot(shape, spacing, origin, so, nbl, dt, nt, vp, src, wav, rec,
                name=f"serving {n}^3 nt={nt}")
    return shot, vp_true
