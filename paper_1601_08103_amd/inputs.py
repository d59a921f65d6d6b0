"""Seeded synthetic inputs: macroscopic initial fields for the LEE lattice Boltzmann runs.

This module is shared by the tests, the benchmark and the smoke check.  It holds no
lattice-Boltzmann arithmetic: it only draws pulse parameters from a seeded PCG64 stream
and evaluates Gaussian / plane-wave fields.  The constants of the target gas (rho0,
theta0, gamma) are passed in by the caller.

Initial-condition modes (the paper starts every run at equilibrium from macroscopic
fields; its Gauss tests put the pulse in the density with theta' = 0):

* "isentropic": a pure acoustic field from a pressure perturbation p'0:
      rho' = p'0 / c^2,  theta' = (gamma - 1) theta0 rho' / rho0,  u' = given (default 0),
  with c^2 = gamma theta0 the LEE sound speed squared.
* "paper": the paper's Gauss-pulse form: rho' = p'0 / theta0, theta' = 0, u' = 0.

Distances are periodic minimum-image distances; sigma is a standard deviation in cells.
Arrays are C-ordered (z, y, x) / (y, x) / (x,), float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Pulse:
    centre: tuple  # (x, y, z) in cells
    amplitude: float
    sigma: float


def _min_image(coord: np.ndarray, c: float, n: int) -> np.ndarray:
    d = coord - c
    return d - n * np.round(d / n)


def gaussian_pressure(shape, pulses) -> np.ndarray:
    """sum_k A_k exp(-|x - x_k|^2 / (2 sigma_k^2)) with periodic minimum-image distance."""
    shape = tuple(int(s) for s in shape)
    dims = list(reversed(shape))  # (nx[, ny[, nz]])
    out = np.zeros(shape)
    for pl in pulses:
        factors = []
        for a, n in enumerate(dims):
            d = _min_image(np.arange(n, dtype=np.float64), float(pl.centre[a]), n)
            factors.append(np.exp(-d * d / (2.0 * pl.sigma * pl.sigma)))
        f = factors[0]
        for a in range(1, len(dims)):
            f = np.multiply.outer(factors[a], f)  # outer dims are slower axes
        out += pl.amplitude * f
    return out


def fields_from_pressure(p0: np.ndarray, rho0: float, theta0: float, gamma: float, mode: str = "isentropic",
                         u0: np.ndarray | None = None):
    """(rho', u', theta') for a pressure perturbation p0; u' has shape (D, *p0.shape)."""
    D = p0.ndim
    u = np.zeros((D,) + p0.shape) if u0 is None else np.asarray(u0, dtype=np.float64)
    if mode == "isentropic":
        rho = p0 / (gamma * theta0)
        theta = (gamma - 1.0) * theta0 * rho / rho0
    elif mode == "paper":
        rho = p0 / theta0
        theta = np.zeros_like(p0)
    else:
        raise ValueError(mode)
    return rho, u, theta


def plane_wave_fields(shape, k, A: float, rho0: float, theta0: float, gamma: float, phase0: float = 0.0):
    """Isentropic acoustic plane wave at t = 0 travelling along k: p' = A cos(k.x + phase0),
    u' = khat p' / (rho0 c)."""
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    coords = [grids[D - 1 - a] for a in range(D)]
    k = np.asarray(k, dtype=np.float64)[:D]
    p = A * np.cos(sum(k[a] * coords[a] for a in range(D)) + phase0)
    c = np.sqrt(gamma * theta0)
    khat = k / np.linalg.norm(k)
    u = np.stack([khat[a] * p / (rho0 * c) for a in range(D)])
    rho, _, theta = fields_from_pressure(p, rho0, theta0, gamma, "isentropic")
    return rho, u, theta


# ---------------------------------------------------------------- the workloads
def pulses_1d(n: int = 1024):
    """One pulse, amplitude 1e-3, sigma 20 cells, centred at cell n/2."""
    return [Pulse((n / 2,), 1e-3, 20.0)]


def pulses_2d(seed: int, n: int = 512, count: int = 16):
    """`count` pulses: centres U[0,n)^2, amplitude U(-1e-3, 1e-3), sigma U(8, 24) cells."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, n, size=(count, 2))
    amp = rng.uniform(-1e-3, 1e-3, size=count)
    sig = rng.uniform(8.0, 24.0, size=count)
    return [Pulse(tuple(cen[i]), float(amp[i]), float(sig[i])) for i in range(count)]


def pulses_3d(seed: int, n: int = 256, count: int = 8, amplitude: float = 1e-3, sigma: float = 12.0):
    """`count` pulses: centres U[0,n)^3, fixed amplitude and sigma."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, n, size=(count, 3))
    return [Pulse(tuple(cen[i]), amplitude, sigma) for i in range(count)]


def random_fields(seed: int, shape, D: int, scale: float = 1e-3):
    """Unstructured seeded fields (rho', u', theta') ~ scale * N(0,1): worst case for the stencil,
    every cell and population carries a distinct value."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    rho = scale * rng.standard_normal(shape)
    u = scale * rng.standard_normal((D,) + shape)
    theta = scale * rng.standard_normal(shape)
    return rho, u, theta
