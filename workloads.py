"""Seeded synthetic inputs for the compact-WENO Euler solver, and error norms.

This module serves both the CPU oracle (``oracle/``) and the HIP path
(``paper_1402_5618_amd``); it imports neither and holds none of the scheme's
arithmetic (no reconstruction, flux, limiter or time stepping).  It only
builds initial cell averages, exact reference averages, and norms.

State layout everywhere: structure of arrays, float64,
  1D: ``[3][n]``       components (rho, rho*u, E)
  2D: ``[4][ny][nx]``  components (rho, rho*u, rho*v, E)
  batched 1D: ``[3][sum(n_i)]`` problems packed back to back.

Initial data are *exact cell averages* (Sec. 2.1, definition of the cell
average): smooth data are averaged in closed form, piecewise-constant data
by the length-weighted average of any cell cut by a discontinuity.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_PERIODIC = 0
BC_TRANSMISSIVE = 1
BC_REFLECTIVE = 2


def _sinc(z: float) -> float:
    return 1.0 if z == 0.0 else math.sin(z) / z


def cell_centres(a: float, b: float, n: int) -> np.ndarray:
    h = (b - a) / n
    return a + (np.arange(n) + 0.5) * h


def prim_to_cons_1d(rho, u, p, gamma):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


# ---------------------------------------------------------------- smooth wave
def density_wave_1d(n: int, t: float = 0.0, gamma: float = 1.4) -> np.ndarray:
    """Example 3.1: rho = 1 + 0.2 sin(pi (x - t)), u = 1, p = 1 on periodic [0, 2].

    Cell averages of sin(pi x) over a cell of width h centred at x_j equal
    sinc(pi h / 2) sin(pi x_j); u and p are constant, so rho*u = rho_bar and
    E = p/(gamma-1) + rho_bar/2 exactly.
    """
    h = 2.0 / n
    x = cell_centres(0.0, 2.0, n)
    rho = 1.0 + 0.2 * _sinc(math.pi * h / 2.0) * np.sin(np.pi * (x - t))
    return np.stack([rho, rho * 1.0, 1.0 / (gamma - 1.0) + 0.5 * rho])


def density_wave_2d(nx: int, ny: int, t: float = 0.0, gamma: float = 1.4,
                    vel: float = 0.7) -> np.ndarray:
    """2D analogue on periodic [0, 2]^2: rho = 1 + 0.2 sin(pi (x + y - 2 vel t)),
    u = v = vel, p = 1.  The exact average factorises into two sinc factors."""
    dx, dy = 2.0 / nx, 2.0 / ny
    x = cell_centres(0.0, 2.0, nx)[None, :]
    y = cell_centres(0.0, 2.0, ny)[:, None]
    f = 0.2 * _sinc(math.pi * dx / 2.0) * _sinc(math.pi * dy / 2.0)
    rho = 1.0 + f * np.sin(np.pi * (x + y - 2.0 * vel * t))
    return np.stack([rho, vel * rho, vel * rho,
                     1.0 / (gamma - 1.0) + 0.5 * rho * (2.0 * vel * vel)])


def _smooth_flow_prim(x, y):
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * x) * np.sin(2.0 * np.pi * y)
    u = 0.4 + 0.1 * np.cos(2.0 * np.pi * y)
    v = -0.3 + 0.1 * np.sin(2.0 * np.pi * x)
    p = 1.0 + 0.1 * np.cos(2.0 * np.pi * (x - y))
    return rho, u, v, p


def smooth_flow_2d(nx: int, ny: int, gamma: float = 1.4, quad: int = 6) -> np.ndarray:
    """A smooth, genuinely two-dimensional, nonlinear state on periodic [0, 1]^2:
    rho = 1 + 0.2 sin(2 pi x) sin(2 pi y), u = 0.4 + 0.1 cos(2 pi y),
    v = -0.3 + 0.1 sin(2 pi x), p = 1 + 0.1 cos(2 pi (x - y)).  Cell averages of
    the conserved variables by quad x quad Gauss-Legendre points per cell."""
    xg, wg = np.polynomial.legendre.leggauss(quad)
    dx, dy = 1.0 / nx, 1.0 / ny
    xc = cell_centres(0.0, 1.0, nx)[None, :]
    yc = cell_centres(0.0, 1.0, ny)[:, None]
    U = np.zeros((4, ny, nx))
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            x = xc + 0.5 * a * dx + 0.0 * yc
            y = yc + 0.5 * b * dy + 0.0 * xc
            rho, u, v, p = _smooth_flow_prim(x, y)
            w = 0.25 * wa * wb
            U[0] += w * rho
            U[1] += w * rho * u
            U[2] += w * rho * v
            U[3] += w * (p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v))
    return U


def smooth_flow_2d_divergence(nx: int, ny: int, gamma: float = 1.4, quad: int = 6) -> np.ndarray:
    """Exact cell averages of -(df/dx + dg/dy) for smooth_flow_2d, with f, g the
    Euler fluxes: the face integrals of the pointwise fluxes (quad Gauss points
    per face) divided by the cell size."""
    xg, wg = np.polynomial.legendre.leggauss(quad)
    dx, dy = 1.0 / nx, 1.0 / ny
    xc = cell_centres(0.0, 1.0, nx)
    yc = cell_centres(0.0, 1.0, ny)
    xf = np.arange(nx + 1) * dx
    yf = np.arange(ny + 1) * dy

    def fluxes(x, y):
        rho, u, v, p = _smooth_flow_prim(x, y)
        E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
        f = np.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
        g = np.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])
        return f, g

    Fx = np.zeros((4, ny, nx + 1))
    Gy = np.zeros((4, ny + 1, nx))
    for b, wb in zip(xg, wg):
        f, _ = fluxes(xf[None, :] + 0.0 * yc[:, None], yc[:, None] + 0.5 * b * dy + 0.0 * xf[None, :])
        Fx += 0.5 * wb * f
        _, g = fluxes(xc[None, :] + 0.5 * b * dx + 0.0 * yf[:, None], yf[:, None] + 0.0 * xc[None, :])
        Gy += 0.5 * wb * g
    return -(Fx[:, :, 1:] - Fx[:, :, :-1]) / dx - (Gy[:, 1:, :] - Gy[:, :-1, :]) / dy


# ----------------------------------------------------------- piecewise data
def piecewise_1d(a: float, b: float, n: int, pieces, gamma: float = 1.4) -> np.ndarray:
    """Exact cell averages of piecewise-constant primitive data.

    ``pieces`` is a list of ``(x_lo, x_hi, rho, u, p)``; each cell receives the
    length-weighted average of the conserved states of the pieces it meets.
    """
    h = (b - a) / n
    edges = a + np.arange(n + 1) * h
    out = np.zeros((3, n))
    for (lo, hi, rho, u, p) in pieces:
        cons = prim_to_cons_1d(rho, u, p, gamma)
        overlap = np.clip(np.minimum(edges[1:], hi) - np.maximum(edges[:-1], lo), 0.0, None) / h
        out += overlap[None, :] * cons[:, None]
    return out


def riemann_1d(a, b, n, x0, left, right, gamma=1.4):
    """Two-state Riemann data; ``left``/``right`` are (rho, u, p)."""
    return piecewise_1d(a, b, n, [(a, x0) + tuple(left), (x0, b) + tuple(right)], gamma)


def lax_1d(n: int = 200, gamma: float = 1.4) -> np.ndarray:
    """Example 3.2 (Lax shock tube) on [-5, 5]: (0.445, 0.698, 3.528) |
    (0.5, 0, 0.571), interface at x = 0; run to t = 1.4, Neumann ends."""
    return riemann_1d(-5.0, 5.0, n, 0.0, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), gamma)


def sod_1d(n: int = 100, gamma: float = 1.4) -> np.ndarray:
    """Example 3.3 (Sod shock tube) on [-5, 5], run to t = 2.  The printed
    states, (0.125, 0, 1) | (1, 0, 1), have equal pressures and no velocity
    (a stationary contact only), which contradicts the waves the example
    describes (a left rarefaction, a right contact and shock); the classical
    data of Sod's 1978 survey that the paper cites, (1, 0, 1) | (0.125, 0, 0.1),
    produce them and are used."""
    return riemann_1d(-5.0, 5.0, n, 0.0, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma)


def shu_osher_1d(n: int = 200, gamma: float = 1.4) -> np.ndarray:
    """Example 3.4 (Mach 3 shock / entropy wave) on [-5, 5], run to t = 1.8:
    (3.857143, 2.629369, 10.33333) for x < -4, then rho = 1 + 0.2 sin(5x),
    u = 0, p = 1.  Exact cell averages (the sine integrates in closed form)."""
    h = 10.0 / n
    edges = -5.0 + np.arange(n + 1) * h
    lo, hi = edges[:-1], edges[1:]
    wl = np.clip(np.minimum(hi, -4.0) - lo, 0.0, None)          # length left of -4
    a = np.maximum(lo, -4.0)                                     # right piece [a, hi]
    wr = np.clip(hi - a, 0.0, None)
    sin_int = np.where(wr > 0, (np.cos(5.0 * a) - np.cos(5.0 * hi)) / 5.0, 0.0)
    L = prim_to_cons_1d(3.857143, 2.629369, 10.33333, gamma)
    rho = (wl * L[0] + wr + 0.2 * sin_int) / h
    mom = wl * L[1] / h
    E = (wl * L[2] + wr * (1.0 / (gamma - 1.0))) / h
    return np.stack([rho, mom, E])


def woodward_colella_1d(n: int = 200, gamma: float = 1.4) -> np.ndarray:
    """Example 3.5 (interacting blast waves) on [0, 1], reflective walls, run
    to t = 0.038: p = 1000 | 0.01 | 100 with rho = 1, u = 0."""
    return piecewise_1d(0.0, 1.0, n, [(0.0, 0.1, 1.0, 0.0, 1000.0), (0.1, 0.9, 1.0, 0.0, 0.01),
                                      (0.9, 1.0, 1.0, 0.0, 100.0)], gamma)


def low_density_123_1d(n: int = 400, gamma: float = 1.4) -> np.ndarray:
    """Example 3.6 on [0, 1] (h = 0.0025), run to t = 0.1:
    (1, -2, 0.4) | (1, 2, 0.4)."""
    return riemann_1d(0.0, 1.0, n, 0.5, (1.0, -2.0, 0.4), (1.0, 2.0, 0.4), gamma)


def strong_shock_1d(n: int = 200, gamma: float = 1.4) -> np.ndarray:
    """Example 3.7 on [0, 1], run to t = 2.5e-6: (1, 0, 1e10) | (0.125, 0, 0.1)."""
    return riemann_1d(0.0, 1.0, n, 0.5, (1.0, 0.0, 1e10), (0.125, 0.0, 0.1), gamma)


def leblanc_1d(n: int = 400, gamma: float = 5.0 / 3.0) -> np.ndarray:
    """Example 3.10 on [0, 9] with gamma = 5/3, run to t = 6: (rho, u, e) =
    (1, 0, 0.1) | (1e-3, 0, 1e-7) at x = 3, so p = (gamma - 1) rho e."""
    g = gamma
    return piecewise_1d(0.0, 9.0, n, [(0.0, 3.0, 1.0, 0.0, (g - 1.0) * 1.0 * 0.1),
                                      (3.0, 9.0, 1e-3, 0.0, (g - 1.0) * 1e-3 * 1e-7)], g)


def double_rarefaction_1d(n: int = 4000, gamma: float = 1.4) -> np.ndarray:
    """Example 3.8 on [-1, 1]: (7, -1, 0.2) | (7, +1, 0.2) (right-state sign as
    in the problem's name: two rarefactions moving apart)."""
    return riemann_1d(-1.0, 1.0, n, 0.0, (7.0, -1.0, 0.2), (7.0, 1.0, 0.2), gamma)


def vacuum_blast_1d(n: int = 4000, gamma: float = 1.4, p_bg: float = 1e-10,
                    p_hot: float = 4e3) -> np.ndarray:
    """Near-vacuum blast on [-1, 1]: rho = 1, u = 0, p = p_bg, with p = p_hot in
    the two centre cells (x in [-h, h])."""
    h = 2.0 / n
    return piecewise_1d(-1.0, 1.0, n, [(-1.0, -h, 1.0, 0.0, p_bg), (-h, h, 1.0, 0.0, p_hot),
                                       (h, 1.0, 1.0, 0.0, p_bg)], gamma)


def sedov_planar_1d(h: float = 0.005, gamma: float = 1.4) -> np.ndarray:
    """Example 3.9 on [0, 4]: p = 4e-13 background and 2.56e8 in the interval of
    width h centred at x = 2 (which straddles two cells of a uniform grid)."""
    n = int(round(4.0 / h))
    return piecewise_1d(0.0, 4.0, n, [(0.0, 2.0 - 0.5 * h, 1.0, 0.0, 4e-13),
                                      (2.0 - 0.5 * h, 2.0 + 0.5 * h, 1.0, 0.0, 2.56e8),
                                      (2.0 + 0.5 * h, 4.0, 1.0, 0.0, 4e-13)], gamma)


def sedov_corner_2d(n: int = 1024, extent: float = 1.1, gamma: float = 1.4,
                    p_bg: float = 1e-10, e_blast: float = 0.244816) -> np.ndarray:
    """Quarter-plane Sedov blast on [0, extent]^2: rho = 1, u = v = 0,
    p = p_bg, and total energy e_blast deposited in cell (0, 0)
    (E = e_blast / dx^2 there)."""
    dx = extent / n
    U = np.zeros((4, n, n))
    U[0] = 1.0
    U[3] = p_bg / (gamma - 1.0)
    U[3, 0, 0] = e_blast / (dx * dx)
    return U


# ---------------------------------------------------------- batched ensemble
@dataclasses.dataclass
class Ensemble:
    lengths: np.ndarray      # int64 [nprob]
    offsets: np.ndarray      # int64 [nprob + 1]
    dx: np.ndarray           # float64 [nprob]
    U: np.ndarray            # float64 [3][sum(lengths)]
    left: np.ndarray         # float64 [nprob][3] (rho, u, p)
    right: np.ndarray        # float64 [nprob][3]
    t_end: float


def riemann_ensemble(nprob: int = 4096, seed: int = 1402, n_lo: int = 256, n_hi: int = 4096,
                     gamma: float = 1.4, t_end: float = 0.2) -> Ensemble:
    """Independent 1D Riemann problems on [0, 1] with the interface at 0.5.

    rho log-uniform in [1e-2, 10], u uniform in [-3, 3], p log-uniform in
    [1e-4, 10] on each side, cell counts uniform integers in [n_lo, n_hi].
    """
    rng = np.random.default_rng(seed)
    lengths = rng.integers(n_lo, n_hi + 1, size=nprob).astype(np.int64)

    def states(k):
        rho = 10.0 ** rng.uniform(-2.0, 1.0, size=k)
        u = rng.uniform(-3.0, 3.0, size=k)
        p = 10.0 ** rng.uniform(-4.0, 1.0, size=k)
        return np.stack([rho, u, p], axis=1)

    left = states(nprob)
    right = states(nprob)
    offsets = np.zeros(nprob + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    U = np.empty((3, int(offsets[-1])))
    for i in range(nprob):
        U[:, offsets[i]:offsets[i + 1]] = riemann_1d(0.0, 1.0, int(lengths[i]), 0.5,
                                                    left[i], right[i], gamma)
    return Ensemble(lengths, offsets, 1.0 / lengths.astype(np.float64), U, left, right, t_end)


def ensemble_subset(ens: Ensemble, idx) -> Ensemble:
    idx = np.asarray(idx, dtype=np.int64)
    lengths = ens.lengths[idx]
    offsets = np.zeros(len(idx) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    U = np.concatenate([ens.U[:, ens.offsets[i]:ens.offsets[i + 1]] for i in idx], axis=1)
    return Ensemble(lengths, offsets, ens.dx[idx].copy(), U, ens.left[idx].copy(),
                    ens.right[idx].copy(), ens.t_end)


# ------------------------------------------------------------------- norms
def error_norms(num: np.ndarray, exact: np.ndarray, cell_volume: float):
    """L1 = vol * sum|e|, L2 = sqrt(vol * sum e^2), Linf = max|e| over cells."""
    e = np.abs(np.asarray(num, dtype=np.float64) - np.asarray(exact, dtype=np.float64))
    return (float(cell_volume * e.sum()), float(math.sqrt(cell_volume * (e * e).sum())),
            float(e.max()))


def pressure(U: np.ndarray, gamma: float = 1.4) -> np.ndarray:
    """p = (gamma - 1)(E - |m|^2 / (2 rho)) for 1D [3,...] or 2D [4,...] states."""
    mom2 = sum(U[k] * U[k] for k in range(1, U.shape[0] - 1))
    return (gamma - 1.0) * (U[-1] - 0.5 * mom2 / U[0])


def specific_internal_energy(U: np.ndarray) -> np.ndarray:
    mom2 = sum(U[k] * U[k] for k in range(1, U.shape[0] - 1))
    return U[-1] / U[0] - 0.5 * mom2 / (U[0] * U[0])
