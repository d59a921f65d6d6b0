"""FP64 oracle of the LEE lattice Boltzmann scheme: moments, equilibrium, update, norms.

TEST INFRASTRUCTURE: only tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU library.

Array conventions: spatial arrays are C-ordered (nz, ny, nx) in 3D, (ny, nx) in 2D and
(nx,) in 1D, x fastest.  Populations are (Q, *spatial).  Velocity vectors are
(cx, cy, cz); the velocity of axis a moves index axis -(a+1) of a spatial array.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from .lattices import Lattice


# ---------------------------------------------------------------- moments and equilibrium
def moment_matrix(lat: Lattice) -> np.ndarray:
    """(D+2, Q) map g -> (rho', u'_1..u'_D, theta').

    rho' = sum g_i; u' = sum c_i g_i / rho0; theta' = ((gamma-1) sum (|c|^2+beta)/2 g - theta0 rho')/rho0
    (monoatomic FDVM section; polyatomic temperature in the polyatomic section).
    """
    D, Q = lat.D, lat.Q
    c2 = (lat.c ** 2).sum(axis=1).astype(np.float64)
    M = np.zeros((D + 2, Q))
    M[0] = 1.0
    for a in range(D):
        M[1 + a] = lat.c[:, a] / lat.rho0
    M[D + 1] = ((lat.gamma - 1.0) * 0.5 * (c2 + lat.beta) - lat.theta0) / lat.rho0
    return M


def moments(lat: Lattice, g: np.ndarray) -> dict:
    """rho', u' (D, ...), theta' and p' = rho0 theta' + theta0 rho' (LEE section) of populations g."""
    D = lat.D
    c2 = (lat.c ** 2).sum(axis=1).astype(np.float64)
    rho = np.tensordot(np.ones(lat.Q), g, axes=(0, 0))
    u = np.stack([np.tensordot(lat.c[:, a].astype(np.float64), g, axes=(0, 0)) / lat.rho0 for a in range(D)])
    e = np.tensordot(0.5 * (c2 + lat.beta), g, axes=(0, 0))
    theta = ((lat.gamma - 1.0) * e - lat.theta0 * rho) / lat.rho0
    p = lat.rho0 * theta + lat.theta0 * rho
    return dict(rho=rho, u=u, theta=theta, p=p)


def equilibrium(lat: Lattice, rho, u, theta) -> np.ndarray:
    """g_i^eq = f*_i (a1 rho' + a2 theta' + b c_i.u' + |c_i|^2/2 (c1 rho' + c2 theta')).

    The polyatomic ansatz; with the monoatomic coefficients this is the exact-Maxwellian
    equilibrium of the monoatomic FDVM section.
    """
    rho = np.asarray(rho, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).reshape((lat.D,) + rho.shape)
    out = np.empty((lat.Q,) + rho.shape)
    for i in range(lat.Q):
        ci = lat.c[i]
        cu = sum(float(ci[a]) * u[a] for a in range(lat.D))
        c2 = float((ci ** 2).sum())
        out[i] = lat.fstar[i] * (lat.a1 * rho + lat.a2 * theta + lat.b * cu + 0.5 * c2 * (lat.c1 * rho + lat.c2 * theta))
    return out


def equilibrium_coeff_matrix(lat: Lattice) -> np.ndarray:
    """(Q, D+2) map (rho', u', theta') -> g^eq, read off the equilibrium formula."""
    D, Q = lat.D, lat.Q
    F = np.zeros((Q, D + 2))
    for i in range(Q):
        c2 = float((lat.c[i] ** 2).sum())
        F[i, 0] = lat.fstar[i] * (lat.a1 + 0.5 * c2 * lat.c1)
        for a in range(D):
            F[i, 1 + a] = lat.fstar[i] * lat.b * lat.c[i, a]
        F[i, D + 1] = lat.fstar[i] * (lat.a2 + 0.5 * c2 * lat.c2)
    return F


def equilibrium_matrix(lat: Lattice) -> np.ndarray:
    """E = d g^eq / d g  (Q x Q): equilibrium coefficients composed with the moment map.

    This is the paper's linear form H(tau=1).  It is built from the moment definitions, so
    its momentum block carries the 1/rho0 of u' = sum c g / rho0.
    """
    return equilibrium_coeff_matrix(lat) @ moment_matrix(lat)


def update_matrix(lat: Lattice, tau: float = 0.5) -> np.ndarray:
    """H(tau) = (1 - 1/tau) I + E / tau  (linear form of the LBE update)."""
    return (1.0 - 1.0 / tau) * np.eye(lat.Q) + equilibrium_matrix(lat) / tau


def gamma_matrix(lat: Lattice, k, tau: float = 0.5) -> np.ndarray:
    """Gamma(k) = D(k) H(tau), D_mm = exp(-i k.c_m)  (von Neumann analysis, lattice units)."""
    k = np.zeros(3) + np.asarray(list(k) + [0.0] * (3 - len(k)), dtype=np.float64)
    phase = np.exp(-1j * (lat.c @ k))
    return phase[:, None] * update_matrix(lat, tau)


# ---------------------------------------------------------------- stepping (C oracle)
_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_lbe_steps.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                         dp, dp, ctypes.c_long, ctypes.c_int]
        lib.oracle_lbe_steps.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def spatial_extent(shape):
    """(nx, ny, nz) of a spatial shape in C order."""
    shape = tuple(shape)
    dims = list(reversed(shape)) + [1] * (3 - len(shape))
    return int(dims[0]), int(dims[1]), int(dims[2])


def steps(lat: Lattice, g: np.ndarray, nsteps: int, tau: float = 0.5, nthreads: int = 1, coeffs: dict | None = None) -> np.ndarray:
    """Advance populations g (Q, *spatial) by nsteps periodic LBE steps; returns a new array.

    `coeffs` may override any of fstar, beta, rho0, theta0, gamma, a1, a2, b, c1, c2
    (used only by the tests that plant mistakes in the oracle).
    """
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float64).copy()
    assert g.shape[0] == lat.Q
    nx, ny, nz = spatial_extent(g.shape[1:])
    co = dict(fstar=lat.fstar, beta=lat.beta, rho0=lat.rho0, theta0=lat.theta0, gamma=lat.gamma,
              a1=lat.a1, a2=lat.a2, b=lat.b, c1=lat.c1, c2=lat.c2, c=lat.c)
    if coeffs:
        co.update(coeffs)
    c = np.ascontiguousarray(co["c"], dtype=np.int32)
    fstar = np.ascontiguousarray(co["fstar"], dtype=np.float64)
    beta = np.ascontiguousarray(co["beta"], dtype=np.float64)
    work = np.empty_like(g)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.oracle_lbe_steps(lat.Q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), fstar.ctypes.data_as(dp),
                              beta.ctypes.data_as(dp), co["rho0"], co["theta0"], co["gamma"], co["a1"], co["a2"],
                              co["b"], co["c1"], co["c2"], float(tau), nx, ny, nz, g.ctypes.data_as(dp),
                              work.ctypes.data_as(dp), int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_lbe_steps rejected its arguments")
    return g


def run(lat: Lattice, rho, u, theta, nsteps: int, tau: float = 0.5, nthreads: int = 1) -> np.ndarray:
    """Initial condition at equilibrium (consistency analysis section), then nsteps LBE steps."""
    return steps(lat, equilibrium(lat, rho, u, theta), nsteps, tau=tau, nthreads=nthreads)


# ---------------------------------------------------------------- norms
def weighted_energy(lat: Lattice, g: np.ndarray) -> float:
    """sum_x sum_i g_i^2 / f*_i: the norm in which E is self-adjoint (stability structure, D3Q19 section)."""
    w = (1.0 / lat.fstar).reshape((lat.Q,) + (1,) * (g.ndim - 1))
    return float(np.sum(w * g * g))


def plain_energy(lat: Lattice, g: np.ndarray) -> float:
    """sum_x sum_i g_i^2: the von Neumann L2 norm; conserved when Gamma(k) is unitary."""
    return float(np.sum(g * g))


def l2_space(eta: np.ndarray, dt: float, D: int) -> float:
    """Discrete L2 norm in space: (sum_j |eta_j|^2 dt^D)^(1/2) (Numerical Results section)."""
    return float(np.sqrt(np.sum(np.abs(eta) ** 2) * dt ** D))


def l2_space_time(etas, dt: float, D: int) -> float:
    """Discrete L2 norm over space-time: (sum_t sum_j |eta|^2 dt^(D+1))^(1/2) (Numerical Results section)."""
    s = 0.0
    for eta in etas:
        s += float(np.sum(np.abs(eta) ** 2))
    return float(np.sqrt(s * dt ** (D + 1)))


def rel_l2(x, ref) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm((np.asarray(x, dtype=np.float64) - ref).ravel())
    den = np.linalg.norm(ref.ravel())
    return float(num / den) if den > 0 else float(num)
