"""The paper's own numerical experiments (Section "Numerical Results") on the GPU path, with
closed-form references in place of the paper's third-party finite-volume solutions.

Every experiment is a Gauss pulse in the density (theta' = 0, u' = 0: the paper's initial
conditions) on a periodic box [0, 1) (1D) or [0, 2)^D, node j at x = j dx, dx = dt = L / N; the
library runs in lattice units (one cell per step), so the pulse exp(-a |x - x_c|^2) becomes a
Gaussian of standard deviation sqrt(1 / (2 a)) / dx cells.  The Gaussian is summed over the
periodic images (the smooth periodic field the closed forms evolve; the paper's expression
is not periodic-smooth at the box edge, e^-7 there in 2D).  The exact solution splits into the
acoustic part (pressure pulse theta0 rho'_0: d'Alembert in 1D, the Hankel form in 2D, the
spherical d'Alembert form in 3D) and the stationary entropy mode.  FP64 storage; errors in the
section's discrete L2 norms."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import lbe
from paper_1601_08103_amd import inputs
from tests._gpu import gpu_ok, lattice, say
from tests.test_paper_points import paper_e5_points

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


def _paper_fields(lat, rho_pulse):
    """(rho', u', theta') of the paper's Gauss initial condition: the density pulse, theta' = 0."""
    return inputs.fields_from_pressure(lat.theta0 * rho_pulse, lat.rho0, lat.theta0, lat.gamma, mode="paper")


def _exact(lat, fields, acoustic):
    """Exact fields from the acoustic part's solution (isentropic closed form of the pressure
    pulse) and the initial stationary entropy mode."""
    _, _, s0 = cf.split_state(lat, *fields)
    return cf.join_state(lat, acoustic["p"], acoustic["u"], s0)


def _run(name, shape, fields, steps):
    from paper_1601_08103_amd.lbm import Solver
    sim = Solver(name, "f64", shape, *fields)
    sim.step(steps)
    m = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    sim.close()
    return m


def _slopes(errs, Ns=None):
    """Observed orders between consecutive grids (N doubling unless Ns is given)."""
    if Ns is None:
        return [float(np.log2(errs[i] / errs[i + 1])) for i in range(len(errs) - 1)]
    return [float(np.log(errs[i] / errs[i + 1]) / np.log(Ns[i + 1] / Ns[i])) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("T", [0.5, 1.0, 2.0])
def test_e1_1d_gauss_space_time_error_at_machine_precision(T):
    """1D: D1Q3 (rho0 = 1, theta0 = 1/3), rho' = exp(-100 (x - 1/2)^2) on [0, 1), end times T: the
    space-time L2 error of the density (norm over every step 0..T) is at machine precision for
    every N, since the set's velocities are the LEE's characteristic speeds (the section's
    finding)."""
    from paper_1601_08103_amd.lbm import Solver
    lat = lattice("D1Q3")
    for N in (50, 100, 200, 400):
        dx = 1.0 / N
        x = np.arange(N) * dx
        rho0 = np.exp(-100.0 * (x - 0.5) ** 2)
        fields = _paper_fields(lat, rho0)
        steps = int(round(T / dx))
        say("E1", T, N, steps)
        sim = Solver("D1Q3", "f64", (N,), *fields)
        errs, refs = [], []
        for n in range(steps + 1):
            if n:
                sim.step(1)
            rho = sim.moments()["rho"].cpu().numpy()
            ex = cf.dalembert_1d_integer_shift(lat, *fields, n)["rho"]
            errs.append(rho - ex)
            refs.append(ex)
        sim.close()
        e = lbe.l2_space_time(errs, dx, 1)
        r = lbe.l2_space_time(refs, dx, 1)
        say("E1", T, N, "space-time L2 error", e, "relative", e / r)
        assert e < 1e-12 * r


def _e23(name, N):
    lat = lattice(name)
    dx = 2.0 / N
    sig = np.sqrt(1.0 / 14.0) / dx  # exp(-7 r^2)
    c = (N / 2.0, N / 2.0)
    fields = _paper_fields(lat, cf.gaussian_periodic((N, N), 1.0, sig, c))
    steps = N // 2  # t = 1
    m = _run(name, (N, N), fields, steps)
    ex = _exact(lat, fields, cf.radial_2d_gaussian(lat, lat.theta0, sig, c, (N, N), float(steps)))
    return {k: lbe.l2_space(m[k] - ex[k], dx, 2) for k in ("rho", "u", "theta", "p")}


@pytest.mark.parametrize("name", ["D2Q5", "D2Q5_DIA"])
def test_e2_e3_2d_gauss_second_order(name):
    """2D: D2Q5 monoatomic (rho0 = 1, theta0 = 1/4) and diatomic (rho0 = 20/3, theta0 = 3/10),
    rho' = exp(-7 |x - (1,1)|^2) on [0, 2)^2, t = 1, N = 32 ... 512: the L2 errors of the
    macroscopic variables against the Hankel solution fall at second order."""
    errs = {k: [] for k in ("rho", "u", "theta", "p")}
    for N in (32, 64, 128, 256, 512):
        say("E2/E3", name, N)
        e = _e23(name, N)
        for k in errs:
            errs[k].append(e[k])
    for k, e in errs.items():
        s = _slopes(e)
        say("E2/E3", name, k, ["%.3e" % v for v in e], ["%.3f" % v for v in s])
        assert min(s[1:]) > 1.9 and max(s) < 2.1, (k, s)


def _e3d(name, N, steps, sig_x=np.sqrt(1.0 / 30.0)):
    lat = lattice(name)
    dx = 2.0 / N
    sig = sig_x / dx  # exp(-15 r^2)
    c = (N / 2.0,) * 3
    fields = _paper_fields(lat, cf.gaussian_periodic((N, N, N), 1.0, sig, c))
    m = _run(name, (N, N, N), fields, steps)
    ex = _exact(lat, fields, cf.radial_3d_gaussian(lat, lat.theta0, sig, c, (N, N, N), float(steps)))
    return m, ex, lat, fields, sig, c


@pytest.mark.parametrize("name", ["D3Q7", "D3Q7_DIA"])
def test_e4_e6_3d_gauss_second_order(name):
    """3D: D3Q7 monoatomic (theta0 = 1/5) and diatomic (f1 = 5/42, theta0 = 5/21),
    rho' = exp(-15 |x - (1,1,1)|^2) on [0, 2)^3, t = 2 (N steps), N = 40, 80, 160: the L2 errors
    of the macroscopic variables against the spherical d'Alembert solution fall at second order."""
    errs = {k: [] for k in ("rho", "u", "p")}
    for N in (40, 80, 160):
        say("E4/E6", name, N)
        m, ex, *_ = _e3d(name, N, N)
        for k in errs:
            errs[k].append(lbe.l2_space(m[k] - ex[k], 2.0 / N, 3))
    for k, e in errs.items():
        s = _slopes(e)
        say("E4/E6", name, k, ["%.3e" % v for v in e], ["%.3f" % v for v in s])
        assert min(s) > 1.9, (k, s)


def test_e5_3d_diatomic_dimensional(golden_dir):
    """3D diatomic, dimensional background rho0 = theta0 = 1 on [0, 2)^3 to dimensional time 1:
    the product's dimensional mapping gives the non-dimensional end time sqrt(21/5) and, for
    N = 25, 40, 80, 120 cells per axis, N_TS = round(T / dt) steps (Table 1).  The density error
    at the end of the run, against the exact solution at the time the run reaches (N_TS dt), falls
    at second order; against the exact solution at T (the paper's comparison, which includes the
    end-time offset of Table 1) it is reported alongside."""
    from paper_1601_08103_amd import lbm
    s = lbm.lbm_lee_dimensional_scaling("D3Q7_DIA", 1.0, 1.0, 1.0)
    e_run, e_T = [], []
    for N in (25, 40, 80, 120):  # the grids of Table 1
        dt = 2.0 / N
        n, t_end, off = lbm.lbm_lee_dimensional_steps(s, 1.0, dt)
        say("E5", N, "steps", n, "offset", off)
        m, ex, lat, fields, sig, c = _e3d("D3Q7_DIA", N, n)
        e_run.append(lbe.l2_space(m["rho"] - ex["rho"], dt, 3))
        T = 1.0 / s.t_star
        exT = _exact(lat, fields, cf.radial_3d_gaussian(lat, lat.theta0, sig, c, (N, N, N), T / dt))
        e_T.append(lbe.l2_space(m["rho"] - exT["rho"], dt, 3))
    Ns = (25, 40, 80, 120)
    say("E5 density error at N_TS dt", ["%.3e" % v for v in e_run], ["%.3f" % v for v in _slopes(e_run, Ns)])
    say("E5 density error at T", ["%.3e" % v for v in e_T], ["%.3f" % v for v in _slopes(e_T, Ns)])
    assert min(_slopes(e_run, Ns)) > 1.9, e_run
    assert all(b < a for a, b in zip(e_T, e_T[1:]))
    # the paper's points (against a finite-volume reference, at the same comparison time T) agree in
    # size: within a factor 1.5 on every grid (measured: 1.04 to 1.30)
    _, _, paper = paper_e5_points(golden_dir)
    say("E5 paper points", ["%.3e" % v for v in paper], "ratio", ["%.2f" % (a / b) for a, b in zip(e_T, paper)])
    for a, b in zip(e_T, paper):
        assert b / 1.5 < a < 1.5 * b, (e_T, paper)
