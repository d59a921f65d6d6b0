"""Closed-form references for the oracle's own pins (none of them runs the stepper).

TEST INFRASTRUCTURE: only tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module.

All quantities are in lattice units (dx = dt = 1).  The LEE without background velocity
(non-dimensional form, LEE section) split into an acoustic part and a stationary part:

  p' = rho0 theta' + theta0 rho'        obeys  d_t p' = -gamma rho0 theta0 div u',
  rho0 d_t u' = -grad p',               so p' solves the wave equation with c^2 = gamma theta0;
  s  = theta' - (gamma-1) theta0 rho' / rho0   obeys d_t s = 0 (it does not move).

Given p' and s:  rho' = (p' - rho0 s) / c^2,  theta' = s + (gamma-1) theta0 rho' / rho0.
"""
from __future__ import annotations

import numpy as np

from .lattices import Lattice
from .lbe import gamma_matrix


def split_state(lat: Lattice, rho, u, theta):
    """(p', u', s) of macroscopic fields."""
    p = lat.rho0 * np.asarray(theta) + lat.theta0 * np.asarray(rho)
    s = np.asarray(theta) - (lat.gamma - 1.0) * lat.theta0 * np.asarray(rho) / lat.rho0
    return p, np.asarray(u), s


def join_state(lat: Lattice, p, u, s):
    """(rho', u', theta') from (p', u', s)."""
    rho = (p - lat.rho0 * s) / lat.cs2
    theta = s + (lat.gamma - 1.0) * lat.theta0 * rho / lat.rho0
    return dict(rho=rho, u=u, theta=theta, p=p)


def dalembert_1d_integer_shift(lat: Lattice, rho, u, theta, n: int):
    """Exact 1D LEE solution on a periodic grid after time n, when c * n is a whole number of cells.

    d'Alembert: p'(x,t) = (P(x-ct) + P(x+ct))/2 + rho0 c (U(x-ct) - U(x+ct))/2,
                u'(x,t) = (U(x-ct) + U(x+ct))/2 + (P(x-ct) - P(x+ct))/(2 rho0 c),
    with P, U the initial p', u' and the stationary s unchanged.  Sampling a shifted grid
    function is exact here because the shift is an integer number of cells.
    """
    c = np.sqrt(lat.cs2)
    shift = c * n
    m = int(round(shift))
    if abs(shift - m) > 1e-12:
        raise ValueError("c*n must be an integer for the sampled d'Alembert solution")
    P, U, S = split_state(lat, rho, np.asarray(u).reshape(-1), theta)
    Pm, Pp = np.roll(P, m), np.roll(P, -m)  # P(x - ct), P(x + ct)
    Um, Up = np.roll(U, m), np.roll(U, -m)
    p = 0.5 * (Pm + Pp) + 0.5 * lat.rho0 * c * (Um - Up)
    uu = 0.5 * (Um + Up) + (Pm - Pp) / (2.0 * lat.rho0 * c)
    return join_state(lat, p, uu[None, :], S)


def plane_wave_continuum(lat: Lattice, k, A: float, shape, t: float, phase0: float = 0.0):
    """Isentropic acoustic plane wave travelling along k:  p' = A cos(k.x - c|k| t + phase0),
    u' = khat p'/(rho0 c), rho' = p'/c^2, theta' = (gamma-1) theta0 rho'/rho0 (s = 0)."""
    k = np.asarray(k, dtype=np.float64)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    # spatial arrays are C-ordered (z, y, x): grid axis -(a+1) is coordinate a
    coords = [grids[len(shape) - 1 - a] for a in range(lat.D)]
    kx = sum(k[a] * coords[a] for a in range(lat.D))
    c = np.sqrt(lat.cs2)
    kn = float(np.linalg.norm(k[: lat.D]))
    p = A * np.cos(kx - c * kn * t + phase0)
    khat = k[: lat.D] / kn
    u = np.stack([khat[a] * p / (lat.rho0 * c) for a in range(lat.D)])
    return join_state(lat, p, u, np.zeros_like(p))


def plane_wave_discrete(lat: Lattice, k, ghat0, shape, n: int, tau: float = 0.5) -> np.ndarray:
    """Populations after n steps of a single Fourier mode: Re(Gamma(k)^n ghat0 exp(i k.x)).

    Von Neumann analysis: the Fourier transform of the linear update is
    ghat(t+1) = Gamma(k) ghat(t), Gamma = D(k) H(tau).  k must be a grid wave vector
    (2 pi m / N per axis) for the periodic box to carry the mode.
    """
    G = gamma_matrix(lat, k, tau)
    gh = np.linalg.matrix_power(G, int(n)) @ np.asarray(ghat0, dtype=np.complex128)
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape], indexing="ij")
    coords = [grids[len(shape) - 1 - a] for a in range(lat.D)]
    kk = np.asarray(list(k) + [0.0] * 3, dtype=np.float64)
    phase = np.exp(1j * sum(kk[a] * coords[a] for a in range(lat.D)))
    return np.real(gh.reshape((-1,) + (1,) * len(shape)) * phase[None])


def radial_3d_gaussian(lat: Lattice, A: float, sigma: float, centre, shape, t: float, images: int | None = None):
    """Isentropic 3D Gaussian pressure pulse p'0 = A exp(-r^2/(2 sigma^2)), u'0 = 0, at time t.

    Spherical d'Alembert solution with f(s) = s P(s) odd:
      p'(r,t) = (f(r - ct) + f(r + ct)) / (2r),   p'(0,t) = P(ct)(1 - (ct)^2/sigma^2);
      u'_r    = -(1/(2 rho0 c)) [ (f(r+ct) - f(r-ct))/r + sigma^2 (P(r+ct) - P(r-ct))/r^2 ],
    obtained from rho0 d_t u' = -grad p' with the antiderivative Phi(s) = -sigma^2 P(s) of f.
    The periodic box is handled by summing periodic images.
    """
    nz, ny, nx = shape
    L = np.array([nx, ny, nz], dtype=np.float64)
    c = np.sqrt(lat.cs2)
    ct = c * t
    reach = ct + 9.0 * sigma
    if images is None:
        images = int(np.ceil(reach / L.min())) + 1
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    P = lambda s: A * np.exp(-s * s / (2.0 * sigma * sigma))
    p = np.zeros(shape)
    u = np.zeros((3,) + tuple(shape))
    rng = range(-images, images + 1)
    for iz in rng:
        for iy in rng:
            for ix in rng:
                cx = centre[0] + ix * L[0]
                cy = centre[1] + iy * L[1]
                cz = centre[2] + iz * L[2]
                dx, dy, dz = x - cx, y - cy, z - cz
                r = np.sqrt(dx * dx + dy * dy + dz * dz)
                if r.min() > reach:
                    continue
                small = r < 1e-9
                rs = np.where(small, 1.0, r)
                pp = ((rs - ct) * P(rs - ct) + (rs + ct) * P(rs + ct)) / (2.0 * rs)
                pp = np.where(small, P(ct) * (1.0 - ct * ct / (sigma * sigma)), pp)
                ur = -(1.0 / (2.0 * lat.rho0 * c)) * (((rs + ct) * P(rs + ct) - (rs - ct) * P(rs - ct)) / rs
                                                      + sigma * sigma * (P(rs + ct) - P(rs - ct)) / (rs * rs))
                ur = np.where(small, 0.0, ur)
                p += pp
                u[0] += ur * dx / rs
                u[1] += ur * dy / rs
                u[2] += ur * dz / rs
    return join_state(lat, p, u, np.zeros_like(p))


def radial_2d_gaussian(lat: Lattice, A: float, sigma: float, centre, shape, t: float, nodes: int = 1000,
                       table: int = 20000):
    """Isentropic 2D Gaussian pressure pulse p'0 = A exp(-r^2/(2 sigma^2)), u'0 = 0, at time t, on
    the periodic box (the sum over periodic images of the free-space solution).

    The 2D wave equation (c^2 = gamma theta0) in the order-0 Hankel representation:
      p'(r,t)   = int_0^inf P(k) cos(c k t) J0(k r) k dk,  P(k) = A sigma^2 exp(-sigma^2 k^2 / 2)
                  (at t = 0 the Hankel pair of the Gaussian),
      u'_r(r,t) = (1 / (rho0 c)) int_0^inf P(k) sin(c k t) J1(k r) k dk
                  (from rho0 d_t u' = -grad p' and d_r J0(k r) = -k J1(k r)).
    Gauss-Legendre quadrature in k on [0, 12/sigma] (P is below exp(-72) A sigma^2 beyond), on a
    table of radii up to c t + 12 sigma (nothing arrives beyond it), then a cubic spline in r.
    """
    from scipy.interpolate import CubicSpline
    from scipy.special import j0, j1

    ny, nx = shape
    L = np.array([nx, ny], dtype=np.float64)
    c = np.sqrt(lat.cs2)
    reach = c * t + 12.0 * sigma
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    K = 12.0 / sigma
    k = 0.5 * K * (xg + 1.0)
    w = 0.5 * K * wg * A * sigma * sigma * np.exp(-0.5 * sigma * sigma * k * k) * k
    rr = np.linspace(0.0, reach, table)
    kr = np.outer(rr, k)
    prof_p = j0(kr) @ (w * np.cos(c * k * t))
    prof_u = j1(kr) @ (w * np.sin(c * k * t)) / (lat.rho0 * c)
    sp, su = CubicSpline(rr, prof_p), CubicSpline(rr, prof_u)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    p = np.zeros(shape)
    u = np.zeros((2,) + tuple(shape))
    images = int(np.ceil(reach / L.min())) + 1
    for iy in range(-images, images + 1):
        for ix in range(-images, images + 1):
            dx = x - (centre[0] + ix * L[0])
            dy = y - (centre[1] + iy * L[1])
            r = np.sqrt(dx * dx + dy * dy)
            near = r <= reach
            if not near.any():
                continue
            rn = r[near]
            p[near] += sp(rn)
            ur = su(rn)
            safe = np.where(rn > 0, rn, 1.0)
            u[0][near] += np.where(rn > 0, ur * dx[near] / safe, 0.0)
            u[1][near] += np.where(rn > 0, ur * dy[near] / safe, 0.0)
    return join_state(lat, p, u, np.zeros_like(p))


def gaussian_periodic(shape, A: float, sigma: float, centre) -> np.ndarray:
    """A exp(-r^2/(2 sigma^2)) summed over the periodic images of the box (C-order shape, centre in
    cells (x, y[, z])): the smooth periodic initial field the radial closed forms evolve."""
    dims = list(reversed([int(s) for s in shape]))
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    coords = [grids[len(shape) - 1 - a] for a in range(len(shape))]
    out = np.zeros(tuple(shape))
    reach = 12.0 * sigma
    rng = [range(-(int(np.ceil(reach / n)) + 1), int(np.ceil(reach / n)) + 2) for n in dims]
    from itertools import product
    for img in product(*rng):
        r2 = sum((coords[a] - (centre[a] + img[a] * dims[a])) ** 2 for a in range(len(dims)))
        out += A * np.exp(-r2 / (2.0 * sigma * sigma))
    return out


def nondimensional_time(t_dim: float, theta0_dim: float, theta0: float, x_star: float = 1.0) -> float:
    """Non-dimensional time for a dimensional one (conversions of the LEE section):
    theta0_dim = theta0* theta0, (u*)^2 = theta0*, u* = x*/t*, t = t_dim / t*."""
    theta_star = theta0_dim / theta0
    u_star = np.sqrt(theta_star)
    t_star = x_star / u_star
    return t_dim / t_star


def end_time_offset(T: float, N: int, length: float = 2.0):
    """(N_TS, T - N_TS dt) for dt = length/N and N_TS = round(T/dt) (Table 1 arithmetic)."""
    dt = length / N
    nts = int(round(T / dt))
    return nts, T - nts * dt
