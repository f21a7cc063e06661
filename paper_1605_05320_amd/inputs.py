"""Seeded synthetic inputs for the shallow-water / adjoint-flagging workloads.

This module only draws random numbers and evaluates analytic bathymetry and
source shapes on grids. It holds none of the method's arithmetic (no Riemann
solver, no limiter, no flagging), so both the HIP library and the CPU oracle
can be fed from it without sharing any numerical code.

The paper's own workload (a trans-Pacific tsunami over ETOPO1 bathymetry,
Section 6) needs data that is not available here; the synthetic basin family
below stands in for it.  Its shape follows the paper's setting: a ~4000 m
abyssal plain, a continental shelf, dry land on one side, an initial hump of
sea surface well offshore and a coastal target region on the shelf.

Conventions
-----------
* Domain [0, L] x [0, L] in metres, x runs west -> east, the coast is on the
  east side.  Cell (i, j) has centre (x_lo + (i + 1/2) dx, y_lo + (j + 1/2) dy).
* Arrays are float64, row-major with x fastest: shape (ny, nx).
* Random draws use numpy's PCG64 (``default_rng(seed)``) in the order listed in
  each function's docstring, so a seed fixes the input completely.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

L_BASIN = 1024.0e3          # basin side (m)
N_SEAMOUNTS = 20


@dataclass
class BasinParams:
    """Random parameters of one member of the synthetic basin family."""
    L: float
    seamounts: np.ndarray            # (20, 4): x_k, y_k, sigma_k, H_k
    src_x: float
    src_y: float
    src_theta: float
    src_amp: float = 1.0
    src_a: float = 0.0               # e-folding half-axes of the elliptical source (m)
    src_b: float = 0.0
    target_xc: float = 0.0
    target_yc: float = 0.0
    target_R: float = 20.0e3
    seed: int = 0


def basin_params(seed: int, L: float = L_BASIN) -> BasinParams:
    """Draw the basin parameters.

    Draw order: for each of the 20 seamounts (x_k ~ U[0.05L, 0.75L],
    y_k ~ U[0.05L, 0.95L], sigma_k ~ U[0.01L, 0.04L], H_k ~ U[500, 2500] m),
    then the source centre (x_s ~ U[0.2L, 0.5L], y_s ~ U[0.3L, 0.7L]) and its
    orientation theta ~ U[0, pi).
    """
    rng = np.random.default_rng(seed)
    sm = np.empty((N_SEAMOUNTS, 4))
    for k in range(N_SEAMOUNTS):
        sm[k, 0] = rng.uniform(0.05 * L, 0.75 * L)
        sm[k, 1] = rng.uniform(0.05 * L, 0.95 * L)
        sm[k, 2] = rng.uniform(0.01 * L, 0.04 * L)
        sm[k, 3] = rng.uniform(500.0, 2500.0)
    xs = rng.uniform(0.2 * L, 0.5 * L)
    ys = rng.uniform(0.3 * L, 0.7 * L)
    th = rng.uniform(0.0, math.pi)
    return BasinParams(L=L, seamounts=sm, src_x=xs, src_y=ys, src_theta=th,
                       src_amp=1.0, src_a=0.08 * L, src_b=0.025 * L,
                       target_xc=0.90 * L, target_yc=0.5 * L, target_R=20.0e3,
                       seed=seed)


def bathymetry(x: np.ndarray, y: np.ndarray, p: BasinParams) -> np.ndarray:
    """Bottom elevation B(x, y) (m, negative below sea level).

    Abyssal plain at -4000 m rising through a tanh shelf break (centred at
    0.85L, width 0.015L) to a -100 m shelf, a linear beach from 0.93L that
    crosses sea level near 0.9475L, plus the Gaussian seamounts.
    """
    L = p.L
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    b0 = -4000.0 + 3900.0 * 0.5 * (1.0 + np.tanh((x - 0.85 * L) / (0.015 * L)))
    bl = np.maximum(0.0, x - 0.93 * L) * (400.0 / (0.07 * L))
    b = b0 + bl
    for xk, yk, sk, hk in p.seamounts:
        b = b + hk * np.exp(-((x - xk) ** 2 + (y - yk) ** 2) / (2.0 * sk * sk))
    return b


def source_surface(x: np.ndarray, y: np.ndarray, p: BasinParams) -> np.ndarray:
    """Initial sea-surface elevation: an elliptical Gaussian hump (1 m peak)."""
    c, s = math.cos(p.src_theta), math.sin(p.src_theta)
    dx = np.asarray(x, dtype=np.float64) - p.src_x
    dy = np.asarray(y, dtype=np.float64) - p.src_y
    xi = c * dx + s * dy
    ze = -s * dx + c * dy
    return p.src_amp * np.exp(-(xi / p.src_a) ** 2 - (ze / p.src_b) ** 2)


@dataclass
class Grid2D:
    nx: int
    ny: int
    dx: float
    dy: float
    x_lo: float = 0.0
    y_lo: float = 0.0

    def centres(self):
        xc = self.x_lo + (np.arange(self.nx) + 0.5) * self.dx
        yc = self.y_lo + (np.arange(self.ny) + 0.5) * self.dy
        return np.meshgrid(xc, yc)          # (ny, nx) each


@dataclass
class Basin2D:
    grid: Grid2D
    B: np.ndarray
    eta0: np.ndarray
    params: BasinParams
    target: tuple = field(default=(0.0, 0.0, 0.0))


def basin(n: int, seed: int, L: float = L_BASIN, ny: int | None = None) -> Basin2D:
    """Synthetic basin on an n x n (or n x ny) grid covering [0, L]^2."""
    ny = n if ny is None else ny
    p = basin_params(seed, L)
    g = Grid2D(nx=n, ny=ny, dx=L / n, dy=L / ny)
    X, Y = g.centres()
    return Basin2D(grid=g, B=bathymetry(X, Y, p), eta0=source_surface(X, Y, p),
                   params=p, target=(p.target_xc, p.target_yc, p.target_R))


# --------------------------------------------------------------------------
# One-dimensional linearized workload (depth ramp towards a shelf).
# --------------------------------------------------------------------------
@dataclass
class Shelf1D:
    nx: int
    dx: float
    x_lo: float
    B: np.ndarray
    eta0: np.ndarray
    x0: float
    target: tuple


def shelf1d(n: int = 2000, seed: int = 0, x_lo: float = -400.0e3, x_hi: float = 0.0,
            step: bool = False, x0: float | None = None, width: float = 10.0e3,
            amp: float = 0.4) -> Shelf1D:
    """1D ocean of depth 4000 m shoaling to a 200 m shelf over the last 50 km.

    ``step=False``: depth 4000 m for x <= -50 km, then linear to 200 m at x = 0.
    ``step=True``: the paper's piecewise-constant variant (4000 m, then 200 m for
    the last 50 km).  Initial surface: amp * exp(-((x - x0)/width)^2) with
    x0 ~ U[-350 km, -100 km] drawn from ``seed`` unless given.
    Target: Gaussian centred 17.5 km offshore with e-folding width 7.5 km.
    """
    rng = np.random.default_rng(seed)
    if x0 is None:
        x0 = rng.uniform(-350.0e3, -100.0e3)
    dx = (x_hi - x_lo) / n
    x = x_lo + (np.arange(n) + 0.5) * dx
    if step:
        depth = np.where(x > -50.0e3, 200.0, 4000.0)
    else:
        frac = np.clip((x + 50.0e3) / 50.0e3, 0.0, 1.0)
        depth = 4000.0 + (200.0 - 4000.0) * frac
    B = -depth
    eta0 = amp * np.exp(-((x - x0) / width) ** 2)
    return Shelf1D(nx=n, dx=dx, x_lo=x_lo, B=B, eta0=eta0, x0=x0,
                   target=(-17.5e3, 0.0, 7.5e3))


# --------------------------------------------------------------------------
# Batched AMR level: many uneven patches cut out of one basin.
# --------------------------------------------------------------------------
@dataclass
class PatchSet:
    nx: np.ndarray        # (P,) int
    ny: np.ndarray
    dx: np.ndarray        # (P,) float
    x_lo: np.ndarray
    y_lo: np.ndarray
    B: list               # list of (ny_p, nx_p) arrays
    eta0: list


def patches(n_patches: int = 3000, seed: int = 4, L: float = L_BASIN,
            nmin: int = 8, nmax: int = 64, base_dx: float = 1.0e3) -> PatchSet:
    """Patches with sides ~ U{nmin..nmax}, dx = base_dx / r with r ~ U{1, 2, 4},
    origins uniform inside the basin; B and the source are sampled from the
    basin family of ``seed`` at the patch cell centres.

    Draw order: the basin parameters (as ``basin_params(seed)``) first, then
    from a second stream ``default_rng(seed + 7919)`` per patch:
    nx_p, ny_p, r, x_lo, y_lo.
    """
    p = basin_params(seed, L)
    rng = np.random.default_rng(seed + 7919)
    nxs = np.empty(n_patches, np.int64)
    nys = np.empty(n_patches, np.int64)
    dxs = np.empty(n_patches)
    xl = np.empty(n_patches)
    yl = np.empty(n_patches)
    Bs, Es = [], []
    for k in range(n_patches):
        nxs[k] = rng.integers(nmin, nmax + 1)
        nys[k] = rng.integers(nmin, nmax + 1)
        r = (1, 2, 4)[rng.integers(0, 3)]
        dxs[k] = base_dx / r
        xl[k] = rng.uniform(0.0, L - nxs[k] * dxs[k])
        yl[k] = rng.uniform(0.0, L - nys[k] * dxs[k])
        g = Grid2D(nx=int(nxs[k]), ny=int(nys[k]), dx=dxs[k], dy=dxs[k],
                   x_lo=xl[k], y_lo=yl[k])
        X, Y = g.centres()
        Bs.append(bathymetry(X, Y, p))
        Es.append(source_surface(X, Y, p))
    return PatchSet(nx=nxs, ny=nys, dx=dxs, x_lo=xl, y_lo=yl, B=Bs, eta0=Es)


# --------------------------------------------------------------------------
# Serving trace: Poisson arrivals of scenarios of different sizes.
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float        # seconds after trace start
    n: int                # grid side
    seed: int


def arrivals(n_requests: int, rate: float, nmin: int = 256, nmax: int = 2048,
             seed: int = 1000) -> list:
    """Poisson trace: exponential inter-arrival gaps with mean 1/rate seconds,
    grid side n ~ U{nmin..nmax}; scenario id k uses basin seed 1000 + k."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(rng.integers(nmin, nmax + 1))
        out.append(Request(rid=k, arrival=t, n=n, seed=1000 + k))
    return out
