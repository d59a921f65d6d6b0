"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import os
import sys

import numpy as np

from oracle import lattices as L
from oracle import lbe


def gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def say(*a):
    """Name the case before GPU work starts, flushed, so a crash still leaves it in the log."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def oracle_threads():
    return int(os.environ.get("LBM_ORACLE_THREADS", str(min(16, os.cpu_count() or 1))))


def oracle_pull_state(lat, t0, n, tau=0.5):
    """Post-collision ("pull") state after n steps from post-collision state t0.

    The library stores g* = H g (collided, not yet streamed); the oracle's push stepper stores
    g (streamed, not yet collided).  With s0 = H^{-1} t0 the oracle's s_n satisfies
    t_n = H s_n.  H(1/2) is its own inverse.
    """
    H = lbe.update_matrix(lat, tau)
    Hinv = np.linalg.inv(H)
    s0 = np.tensordot(Hinv, t0, axes=(1, 0))
    sn = lbe.steps(lat, s0, n, tau=tau, nthreads=oracle_threads())
    return np.tensordot(H, sn, axes=(1, 0))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (d if d > 0 else 1.0))


def stable_seed(*parts):
    import zlib
    return zlib.crc32(repr(parts).encode())


def lattice(name):
    return L.get(name)
