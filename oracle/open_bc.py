"""FP64 reference of the open-boundary closures (not in the paper: it treats periodic domains
only and leaves boundary conditions to future work).

TEST INFRASTRUCTURE: only tests, the package smoke check and the benchmark's CPU-baseline
leg may import this module.

Definitions (these are the build's own, stated here and nowhere else in code):

State.  The post-collision populations g*(x) on the box [0, n_a) per axis ("pull" state,
the same convention as the GPU library).  One step: for every cell x and population i the
streamed value is g*_i(x - c_i) when x - c_i is inside the box, else a ghost value given by
the closure; then the collision (the paper's LBE relaxation) at x; then, for the sponge, a
damping of the new post-collision values near the faces.

Closures for a source s = x - c_i outside the box:
  "zero"    0 (the exterior is at rest),
  "copy"    g*_i(clamp(s)) (zero normal gradient; clamp = nearest cell of the box),
  "sponge"  0, and after the collision g* <- (1 - sigma(d)) g* for cells at distance
            d = min_a min(x_a, n_a - 1 - x_a) < W from the faces, sigma(d) = sigma_max ((W-d)/W)^2,
  "mlp"     a network prediction (below); with a width W >= 1 given, the new post-collision
            values are then damped as the sponge damps them (a network behind a sponge layer),
  "external" the value of a given outer state at s (a test device: with the state of a
            larger periodic run the open step must reproduce that run inside the box).

Faces and the canonical frame.  Face (a, side): axis a, side 0 = low (x_a = 0), 1 = high.
p = clamp(s) is the face node.  A source outside along one axis takes that face's
prediction at p; a source beyond an edge or a corner takes the mean of the predictions of
every face it lies beyond (the same node p), which keeps the closure symmetric under the
box's symmetries.
The network's prediction at p for a face is then limited in energy (weighted norm
sum g^2 / f*, conserved by the collision at tau = 1/2 and by streaming): with E_in the energy
of the k predicted values and E_out that of the populations leaving p through the face
(canonical c'_x = -1), the prediction is scaled by sqrt(B / E_in) when E_in > B, where
B = E_out / (2^n - 1) and n is the number of faces p lies on.  Every ghost value pulled into
the box is attributed to its node p; a face prediction at p feeds the ghost cells beyond
every subset of p's faces that contains the face, at most (2^n - 1) / n times its energy in
total (mean over faces, Jensen), while the populations leaving p carry at least the mean of
the n face energies E_out.  So the energy entering at p never exceeds the energy leaving p,
and the open box's energy cannot grow, whatever the network predicts.
A signed axis permutation M maps the face's outward normal to -x (the canonical face), so
one network serves every face:  (a,0): identity; (a,1): negate axis a; then axis a is
swapped with x.  In the canonical frame the populations that enter through the face are
those with c'_x = +1.  A strip is g*(p + m n_in), m = 0, 1, 2 (n_in the inward normal), listed
m-major with populations in canonical order; the network input is the strip of the current state
followed by the strip of the state one step earlier (the current one again on the first step);
its output is the k entering populations in canonical order.
"""
from __future__ import annotations

import numpy as np

from . import mlp as mlp_ref
from .lattices import Lattice
from .lbe import update_matrix


def faces(D):
    return [(a, side) for a in range(D) for side in (0, 1)]


def face_transform(a: int, side: int) -> np.ndarray:
    """3x3 signed permutation M with M n_out = (-1, 0, 0)."""
    M = np.eye(3, dtype=np.int64)
    if side == 1:
        M[a, a] = -1
    P = np.eye(3, dtype=np.int64)
    P[[0, a]] = P[[a, 0]]  # swap axis a and x
    return P @ M


def canonical_perm(lat: Lattice, a: int, side: int) -> np.ndarray:
    """perm[j] = face population index i whose velocity maps to canonical velocity j."""
    M = face_transform(a, side)
    cc = lat.c @ M.T  # canonical velocities of every population, c' = M c
    perm = np.empty(lat.Q, dtype=np.int64)
    for j in range(lat.Q):
        hits = np.where((cc == lat.c[j]).all(axis=1))[0]
        assert len(hits) == 1
        perm[j] = hits[0]
    return perm


def incoming_canonical(lat: Lattice) -> np.ndarray:
    """Canonical indices j with c'_x = +1, in increasing order."""
    return np.where(lat.c[:, 0] == 1)[0]


def strip(lat: Lattice, g, a: int, side: int, node) -> np.ndarray:
    """Network input (3Q,) at face node `node` (a full spatial index tuple, C order)."""
    perm = canonical_perm(lat, a, side)
    D = lat.D
    ax = D - 1 - a  # array axis of coordinate a
    step = 1 if side == 0 else -1
    vals = []
    for m in range(3):
        idx = list(node)
        idx[ax] += m * step
        cell = tuple(idx)
        vals.append(np.array([g[(perm[j],) + cell] for j in range(lat.Q)]))
    return np.concatenate(vals)


def _clamp(idx, shape):
    return tuple(min(max(v, 0), n - 1) for v, n in zip(idx, shape))


def _out_faces(idx, shape, D):
    """Faces (a, side) beyond which idx lies, in axis order."""
    out = []
    for a in range(D):
        ax = D - 1 - a
        if idx[ax] < 0:
            out.append((a, 0))
        elif idx[ax] >= shape[ax]:
            out.append((a, 1))
    return out


def node_face_count(p, shape, D) -> int:
    """Number of faces the box cell p (C-order index) lies on."""
    n = 0
    for a in range(D):
        ax = D - 1 - a
        n += int(p[ax] == 0) + int(p[ax] == shape[ax] - 1)
    return n


def energy_limit(lat: Lattice, x, y, nfaces: int) -> np.ndarray:
    """Scale the prediction y (k entering values, canonical order) so that its weighted energy
    is at most E_out / (2^nfaces - 1), E_out from the populations of the strip's first cell
    that leave through the face (canonical c'_x = -1)."""
    jin = incoming_canonical(lat)
    jout = np.where(lat.c[:, 0] == -1)[0]
    e_in = float(np.sum(np.asarray(y) ** 2 / lat.fstar[jin]))
    e_out = float(np.sum(np.asarray(x)[jout] ** 2 / lat.fstar[jout]))
    budget = e_out / (2 ** nfaces - 1)
    if e_in > budget:
        return np.asarray(y) * np.sqrt(budget / e_in)
    return np.asarray(y)


def ghost_values(lat: Lattice, g, closure: str, params: dict | None = None, quantize: bool = False,
                 limit: bool = True, g_prev=None):
    """Padded populations (Q, n+2 per axis) whose one-cell shell holds the closure's ghosts.
    The network sees [strip of g, strip of g_prev] (g_prev: the state one step earlier; None on
    the first step, when the current strip stands in for it).  limit=False drops the energy limit
    of the network closure (a test device)."""
    shape = g.shape[1:]
    D = lat.D
    pad = np.zeros((lat.Q,) + tuple(n + 2 for n in shape))
    inner = (slice(None),) + tuple(slice(1, n + 1) for n in shape)
    pad[inner] = g
    if closure in ("zero", "sponge"):
        return pad
    if closure == "external":
        ext = np.asarray(params)  # (Q, n+2 per axis): the outer state around the box
        shell = np.ones(pad.shape[1:], dtype=bool)
        shell[tuple(slice(1, n + 1) for n in shape)] = False
        pad[:, shell] = ext[:, shell]
        return pad
    it = np.ndindex(*pad.shape[1:])
    jin = incoming_canonical(lat) if closure == "mlp" else None
    cache = {}
    for pidx in it:
        s = tuple(v - 1 for v in pidx)
        fs = _out_faces(s, shape, D)
        if not fs:
            continue
        p = _clamp(s, shape)
        if closure == "copy":
            pad[(slice(None),) + pidx] = g[(slice(None),) + p]
        elif closure == "mlp":
            acc = {}
            for a, side in fs:
                key = (a, side, p)
                if key not in cache:
                    x = strip(lat, g, a, side, p)
                    xp = strip(lat, g_prev, a, side, p) if g_prev is not None else x
                    y = mlp_ref.predict(params, np.concatenate([x, xp])[None, :], quantize)[0]
                    cache[key] = energy_limit(lat, x, y, node_face_count(p, shape, D)) if limit else y
                perm = canonical_perm(lat, a, side)
                for r, j in enumerate(jin):
                    acc.setdefault(perm[j], []).append(cache[key][r])
            for i, vals in acc.items():
                # only the populations entering through every listed face are ever pulled
                # from this ghost; others keep 0
                if len(vals) == len(fs):
                    pad[(i,) + pidx] = sum(vals) / len(vals)
        else:
            raise ValueError(closure)
    return pad


def sponge_factor(shape, D, width: int, sigma_max: float) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    d = np.full(shape, np.iinfo(np.int64).max)
    for ax in range(D):
        n = shape[ax]
        d = np.minimum(d, np.minimum(grids[ax], n - 1 - grids[ax]))
    sig = np.where(d < width, sigma_max * ((width - d) / width) ** 2, 0.0)
    return 1.0 - sig


def step_open(lat: Lattice, g, closure: str, tau: float = 0.5, params: dict | None = None,
              sponge_width: int = 0, sponge_sigma: float = 0.0, quantize: bool = False,
              limit: bool = True, g_prev=None) -> np.ndarray:
    """One step of the open-box scheme on the post-collision state g (Q, *shape); g_prev is the
    state one step earlier (the network closure's second time level).  sponge_width: the damped
    layer of the "sponge" closure, and of the "mlp" closure when >= 1 (0: none)."""
    shape = g.shape[1:]
    D = lat.D
    pad = ghost_values(lat, g, closure, params, quantize, limit, g_prev)
    pulled = np.empty_like(g)
    for i in range(lat.Q):
        sl = []
        for ax in range(D):
            a = D - 1 - ax
            c = int(lat.c[i, a])
            sl.append(slice(1 - c, 1 - c + shape[ax]))
        pulled[i] = pad[(i,) + tuple(sl)]
    H = update_matrix(lat, tau)
    out = np.tensordot(H, pulled, axes=(1, 0))
    if closure == "sponge" or (closure == "mlp" and sponge_width >= 1):
        out *= sponge_factor(shape, D, sponge_width, sponge_sigma)[None]
    return out


def run_open(lat: Lattice, g0, nsteps: int, closure: str, **kw) -> np.ndarray:
    g = np.array(g0, dtype=np.float64)
    prev = None
    for _ in range(nsteps):
        g, prev = step_open(lat, g, closure, g_prev=prev, **kw), g
    return g
