"""Velocity sets of the LEE lattice Boltzmann schemes, built in exact rational arithmetic.

TEST INFRASTRUCTURE (part of the oracle): only tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path never does.

Every table is generated from the formulas the paper prints, not typed in as decimals:

* D1Q3: Section "Examples of Velocity Sets", subsection D1Q3 (rho0 = 1, theta0 = 1/3).
* D2Q5 monoatomic: subsection "D2Q5 for Monoatomic Gases" (rho0 = 1, theta0 = 1/4).
* D2Q5 diatomic: subsection "D2Q5 for Diatomic Gases" (rho0 = 20/3, theta0 = 3/10,
  beta, and the coefficients a1, a2, b, c1, c2 printed there).
* 3D monoatomic family f*(rho0, theta0, alpha) on the 27 velocities of Section "3D",
  reduced to D3Q7 (theta0 = 1/5, alpha = 0), D3Q9 (3/5, 3/40), D3Q13 (2/5, 0) and
  D3Q19 (3/10, 0) by dropping the velocities whose weight is zero, and in full as D3Q27
  (1/3, 1/216: every weight positive).
* D3Q7 diatomic family: subsection "Diatomic Gases" of Section "3D" with f1 = 5/42.
* D2Q9 is NOT in the paper.  Its weights are derived here from the similarity
  conditions of Section "Derivation of Finite Discrete Velocity Models for Monoatomic
  Gases" (moments of f* equal those of the Maxwellian for zeta in {1, |v|^2/2,
  v_a v_b, |v|^2 v_a v_b / 2, |v|^4 / 4}) for rest/axis/diagonal weights at theta0 = 1/3:
  w_axis = theta0 (1 - 2 theta0), w_diag = theta0 (4 theta0 - 1) / 4,
  w_rest = 1 - 3 theta0 + 4 theta0^2.

Monoatomic sets use the equilibrium of the monoatomic FDVM section,
g_i^eq = f*_i (rho'/rho0 + c_i.u'/theta0 + theta'(|c_i|^2/(2 theta0^2) - D/(2 theta0))),
which is the general polyatomic form (Section "Generalization ... for Polyatomic Gases")
with a1 = 1/rho0, a2 = -D/(2 theta0), b = 1/theta0, c1 = 0, c2 = 1/theta0^2, beta = 0
and gamma = (D + 2)/D.  Diatomic sets use gamma = (M + 2)/M with M = 2D - 1.

Canonical velocity order (free, see the paper's differing orders): rest first, then
axis velocities (-x, +x, -y, +y, -z, +z), then edges, then corners.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction as Fr
from itertools import product

import numpy as np


@dataclass(frozen=True)
class Lattice:
    name: str
    D: int
    c: np.ndarray  # (Q, 3) int, unused components 0
    fstar: np.ndarray  # (Q,) float64
    beta: np.ndarray  # (Q,) float64
    rho0: float
    theta0: float
    gamma: float
    a1: float
    a2: float
    b: float
    c1: float
    c2: float
    exact: dict = field(default_factory=dict, compare=False, repr=False)

    @property
    def Q(self) -> int:
        return int(self.c.shape[0])

    @property
    def cs2(self) -> float:
        """Squared sound speed of the LEE: gamma * theta0 (from the non-dimensional LEE)."""
        return self.gamma * self.theta0


def _axis_order(D):
    out = []
    for a in range(D):
        for s in (-1, 1):
            v = [0, 0, 0]
            v[a] = s
            out.append(tuple(v))
    return out


def _class_velocities(D, nnz):
    """All velocities in {-1,0,1}^D with exactly nnz non-zero components, deterministic order."""
    out = []
    for v in product((-1, 0, 1), repeat=D):
        if sum(1 for x in v if x != 0) == nnz:
            out.append(tuple(v) + (0,) * (3 - D))
    if nnz == 1:
        return _axis_order(D)
    # order by (position of non-zeros, sign pattern) for readability
    def key(v):
        nzpos = tuple(i for i in range(3) if v[i] != 0)
        return (nzpos, tuple(v[i] for i in nzpos))
    return sorted(out, key=key)


def _mono_coeffs(D, rho0, theta0):
    return dict(a1=1 / rho0, a2=Fr(-D, 2) / theta0, b=1 / theta0, c1=Fr(0), c2=1 / (theta0 * theta0),
                gamma=Fr(D + 2, D))


def _make(name, D, vel_w, rho0, theta0, coeffs, beta_of=None):
    vel_w = [(v, w) for v, w in vel_w if w != 0]  # zero-weight velocities are dropped
    c = np.array([v for v, _ in vel_w], dtype=np.int64)
    f = [w for _, w in vel_w]
    beta = [beta_of(v) if beta_of else Fr(0) for v, _ in vel_w]
    exact = dict(fstar=f, beta=beta, rho0=rho0, theta0=theta0, **coeffs)
    return Lattice(name=name, D=D, c=c, fstar=np.array([float(x) for x in f]),
                   beta=np.array([float(x) for x in beta]), rho0=float(rho0), theta0=float(theta0),
                   gamma=float(coeffs["gamma"]), a1=float(coeffs["a1"]), a2=float(coeffs["a2"]),
                   b=float(coeffs["b"]), c1=float(coeffs["c1"]), c2=float(coeffs["c2"]), exact=exact)


def d1q3():
    rho0, theta0 = Fr(1), Fr(1, 3)
    vw = [((0, 0, 0), Fr(2, 3)), ((-1, 0, 0), Fr(1, 6)), ((1, 0, 0), Fr(1, 6))]
    return _make("D1Q3", 1, vw, rho0, theta0, _mono_coeffs(1, rho0, theta0))


def d2q5():
    rho0, theta0 = Fr(1), Fr(1, 4)
    vw = [((0, 0, 0), Fr(1, 2))] + [(v, Fr(1, 8)) for v in _axis_order(2)]
    return _make("D2Q5", 2, vw, rho0, theta0, _mono_coeffs(2, rho0, theta0))


def d2q9_weights(theta0):
    """Rest/axis/diagonal weights solving the similarity conditions in 2D (rho0 = 1)."""
    w1 = theta0 * (1 - 2 * theta0)
    w2 = theta0 * (4 * theta0 - 1) / 4
    w0 = 1 - 3 * theta0 + 4 * theta0 * theta0
    return w0, w1, w2


def d2q9(theta0=Fr(1, 3)):
    rho0 = Fr(1)
    w0, w1, w2 = d2q9_weights(theta0)
    vw = ([((0, 0, 0), w0)] + [(v, w1) for v in _class_velocities(2, 1)]
          + [(v, w2) for v in _class_velocities(2, 2)])
    return _make("D2Q9", 2, vw, rho0, theta0, _mono_coeffs(2, rho0, theta0))


def d2q5_dia():
    rho0, theta0 = Fr(20, 3), Fr(3, 10)
    vw = [((0, 0, 0), Fr(8, 3))] + [(v, Fr(1)) for v in _axis_order(2)]
    coeffs = dict(a1=1 / rho0, a2=Fr(-5), b=1 / theta0, c1=Fr(0), c2=5 / theta0, gamma=Fr(5, 3))
    return _make("D2Q5_DIA", 2, vw, rho0, theta0, coeffs,
                 beta_of=lambda v: Fr(0) if v == (0, 0, 0) else Fr(1, 2))


def family27_weights(rho0, theta0, alpha):
    """The 27-velocity monoatomic family f*(rho0, theta0, alpha): rest, axis, edge, corner weights."""
    rest = rho0 * theta0 * (15 * theta0 - 9) / 2 + rho0 - 8 * alpha
    axis = rho0 * theta0 * (2 - 5 * theta0) / 2 + 4 * alpha
    edge = rho0 * theta0 * (5 * theta0 - 1) / 8 - 2 * alpha
    corner = alpha
    return rest, axis, edge, corner


def family27(name, theta0, alpha, rho0=Fr(1)):
    rest, axis, edge, corner = family27_weights(rho0, theta0, alpha)
    vw = ([((0, 0, 0), rest)] + [(v, axis) for v in _class_velocities(3, 1)]
          + [(v, edge) for v in _class_velocities(3, 2)] + [(v, corner) for v in _class_velocities(3, 3)])
    return _make(name, 3, vw, rho0, theta0, _mono_coeffs(3, rho0, theta0))


def d3q7():
    return family27("D3Q7", Fr(1, 5), Fr(0))


def d3q9():
    return family27("D3Q9", Fr(3, 5), Fr(3, 40))


def d3q13():
    return family27("D3Q13", Fr(2, 5), Fr(0))


def d3q19():
    return family27("D3Q19", Fr(3, 10), Fr(0))


def d3q27():
    """The member of the 27-velocity family with every weight positive that the build uses:
    theta0 = 1/3, alpha = 1/216 (weights 8/27, 2/27, 1/54, 1/216).  The paper prints the family,
    not this member."""
    return family27("D3Q27", Fr(1, 3), Fr(1, 216))


def d3q7_dia(f1=Fr(5, 42)):
    rho0, theta0 = Fr(42, 5) * f1, Fr(5, 21)
    vw = [((0, 0, 0), Fr(12, 5) * f1)] + [(v, f1) for v in _axis_order(3)]
    coeffs = dict(a1=1 / rho0, a2=Fr(-21, 2), b=Fr(21, 5), c1=Fr(0), c2=Fr(147, 5), gamma=Fr(7, 5))
    return _make("D3Q7_DIA", 3, vw, rho0, theta0, coeffs,
                 beta_of=lambda v: Fr(0) if v == (0, 0, 0) else Fr(2, 3))


ALL = {
    "D1Q3": d1q3, "D2Q5": d2q5, "D2Q9": d2q9, "D3Q7": d3q7, "D3Q9": d3q9, "D3Q13": d3q13,
    "D3Q19": d3q19, "D2Q5_DIA": d2q5_dia, "D3Q7_DIA": d3q7_dia, "D3Q27": d3q27,
}

MONOATOMIC = ("D1Q3", "D2Q5", "D2Q9", "D3Q7", "D3Q9", "D3Q13", "D3Q19", "D3Q27")


def get(name: str) -> Lattice:
    return ALL[name]()
