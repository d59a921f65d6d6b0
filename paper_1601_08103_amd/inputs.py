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


@dataclass(frozen=True)
class Packet:
    centre: tuple     # (x, y, z) in cells
    k: tuple          # wave vector (kx, ky, kz), radians per cell; travels along k
    amplitude: float
    width: float      # Gaussian envelope standard deviation in cells


def packet_fields(shape, packets, rho0: float, theta0: float, gamma: float):
    """Isentropic wave packets p' = A cos(k.(x - x0)) exp(-|x - x0|^2 / (2 w^2)) travelling along
    k (u' = khat p' / (rho0 c), c^2 = gamma theta0).  Plain (not periodic) distances: the packets
    must lie well inside the box."""
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    coords = [grids[D - 1 - a] for a in range(D)]
    c = np.sqrt(gamma * theta0)
    p = np.zeros(shape)
    u = np.zeros((D,) + shape)
    for pk in packets:
        d = [coords[a] - pk.centre[a] for a in range(D)]
        r2 = sum(x * x for x in d)
        kx = sum(pk.k[a] * d[a] for a in range(D))
        pp = pk.amplitude * np.cos(kx) * np.exp(-r2 / (2.0 * pk.width * pk.width))
        kn = float(np.linalg.norm(pk.k[:D]))
        p += pp
        for a in range(D):
            u[a] += (pk.k[a] / kn) * pp / (rho0 * c)
    rho, _, theta = fields_from_pressure(p, rho0, theta0, gamma, "isentropic")
    return rho, u, theta


def random_packets(rng, L: int, D: int, count: int = 1, lam=(16.0, 64.0), amp: float = 1e-3, width_factor=2.0,
                   margin_factor: float = 2.5):
    """`count` packets in an L^D box: wavelength U(lam), width = width_factor * wavelength, centre
    drawn so the envelope (margin_factor widths) stays inside where the box allows it (else the box
    centre), travelling along a uniformly random direction (so it meets the faces at random angles)."""
    out = []
    for _ in range(count):
        lamb = float(rng.uniform(*lam))
        w = width_factor * lamb
        lo, hi = margin_factor * w, L - margin_factor * w
        centre = tuple(float(rng.uniform(lo, hi)) if hi > lo else L / 2.0 for _ in range(D))
        v = rng.standard_normal(D)
        v /= np.linalg.norm(v)
        k = tuple(float(x) * 2.0 * np.pi / lamb for x in v) + (0.0,) * (3 - D)
        out.append(Packet(centre, k, float(rng.choice([-1.0, 1.0])) * amp, w))
    return out


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
