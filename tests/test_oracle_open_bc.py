"""Pins of the open-boundary and network references (CPU only).  The paper has no
boundaries; these definitions are the build's own and are pinned against exact facts:
domain of dependence, energy of a truncated isometry, fixed points, symmetry, and finite
differences for the network gradients."""
import numpy as np
import pytest

from oracle import lattices as L
from oracle import lbe
from oracle import mlp
from oracle import open_bc as ob

from paper_1601_08103_amd import inputs


def _pull_periodic(lat, t0, n, tau=0.5):
    """Periodic pull-state evolution from the oracle's push stepper (t = H s, H(1/2)^2 = I)."""
    H = lbe.update_matrix(lat, tau)
    s0 = np.tensordot(np.linalg.inv(H), t0, (1, 0))
    return np.tensordot(H, lbe.steps(lat, s0, n, tau=tau), (1, 0))


@pytest.mark.parametrize("name", ["D2Q5", "D2Q9", "D3Q7", "D3Q19", "D1Q3"])
def test_external_ghosts_reproduce_the_larger_periodic_run(name):
    lat = L.get(name)
    inner = {1: (20,), 2: (12, 14), 3: (6, 7, 8)}[lat.D]
    outer = tuple(n + 10 for n in inner)
    off = 5
    rng = np.random.default_rng(3)
    big = rng.standard_normal((lat.Q,) + outer)
    box = (slice(None),) + tuple(slice(off, off + n) for n in inner)
    win = (slice(None),) + tuple(slice(off - 1, off + n + 1) for n in inner)
    g = big[box].copy()
    for _ in range(4):
        g = ob.step_open(lat, g, "external", params=big[win])
        big = _pull_periodic(lat, big, 1)
        assert np.abs(g - big[box]).max() < 1e-12 * np.abs(big).max()


@pytest.mark.parametrize("name", ["D2Q9", "D3Q7", "D2Q5"])
def test_zero_closure_never_adds_energy(name):
    """Open box with an exterior at rest = the periodic isometry on an unbounded domain
    followed by truncation: the weighted energy never grows and drops once waves exit."""
    lat = L.get(name)
    shape = {2: (24, 24), 3: (12, 12, 12)}[lat.D]
    p0 = inputs.gaussian_pressure(shape, [inputs.Pulse(tuple(n / 2 for n in shape), 1e-3, 2.0)])
    g = lbe.equilibrium(lat, *inputs.fields_from_pressure(p0, lat.rho0, lat.theta0, lat.gamma))
    E = [lbe.weighted_energy(lat, g)]
    for _ in range(30):
        g = ob.step_open(lat, g, "zero")
        E.append(lbe.weighted_energy(lat, g))
    assert all(E[i + 1] <= E[i] * (1 + 1e-14) for i in range(len(E) - 1))
    assert E[-1] < 0.5 * E[0]


@pytest.mark.parametrize("name", ["D2Q9", "D3Q7"])
def test_copy_closure_keeps_a_uniform_state(name):
    lat = L.get(name)
    shape = {2: (9, 10), 3: (5, 6, 7)}[lat.D]
    g = lbe.equilibrium(lat, np.full(shape, 2e-3), np.full((lat.D,) + shape, 1e-3), np.full(shape, -1e-3))
    out = ob.run_open(lat, g, 5, "copy")
    assert np.abs(out - g).max() < 1e-15


def test_sponge_without_damping_is_the_zero_closure():
    lat = L.get("D2Q9")
    g = np.random.default_rng(1).standard_normal((lat.Q, 16, 18))
    a = ob.step_open(lat, g, "sponge", sponge_width=6, sponge_sigma=0.0)
    b = ob.step_open(lat, g, "zero")
    assert np.array_equal(a, b)
    f = ob.sponge_factor((16, 18), 2, 6, 0.3)
    assert f[8, 9] == 1.0 and abs(f[0, 9] - 0.7) < 1e-15 and abs(f[5, 9] - (1 - 0.3 / 36)) < 1e-15


def _copy_network(lat):
    """Weights that make the network output the m = 0 strip value of each entering population,
    i.e. the copy closure: h = relu(+x), relu(-x); y = h+ - h-."""
    Q = lat.Q
    jin = ob.incoming_canonical(lat)
    k = len(jin)
    p = {"W1": np.zeros((6 * Q, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, k)), "b3": np.zeros(k)}
    for r, j in enumerate(jin):
        p["W1"][j, 2 * r] = 1.0
        p["W1"][j, 2 * r + 1] = -1.0
        p["W2"][2 * r, 2 * r] = 1.0
        p["W2"][2 * r + 1, 2 * r + 1] = 1.0
        p["W3"][2 * r, r] = 1.0
        p["W3"][2 * r + 1, r] = -1.0
    return p


@pytest.mark.parametrize("name", ["D2Q9", "D2Q5", "D3Q7", "D3Q19"])
def test_network_closure_plumbing_against_copy(name):
    """A network that copies the boundary value reproduces the copy closure exactly: this pins
    the canonical frames, the strip layout and the output mapping."""
    lat = L.get(name)
    shape = {2: (7, 9), 3: (4, 5, 6)}[lat.D]
    g = np.random.default_rng(2).standard_normal((lat.Q,) + shape)
    a = ob.step_open(lat, g, "mlp", params=_copy_network(lat), limit=False)
    b = ob.step_open(lat, g, "copy")
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("name", ["D2Q9", "D3Q7"])
def test_network_closure_history_plumbing(name):
    """A network that copies the boundary value of the previous step's strip: its first step
    equals the copy closure (the current strip stands in for the missing history), its second
    step takes the ghosts of the copy closure applied to the state one step earlier."""
    lat = L.get(name)
    Q = lat.Q
    shape = {2: (7, 9), 3: (4, 5, 6)}[lat.D]
    jin = ob.incoming_canonical(lat)
    k = len(jin)
    p = {"W1": np.zeros((6 * Q, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, k)), "b3": np.zeros(k)}
    for r, j in enumerate(jin):  # rows 3Q + j: the earlier strip's first cell
        p["W1"][3 * Q + j, 2 * r] = 1.0
        p["W1"][3 * Q + j, 2 * r + 1] = -1.0
        p["W2"][2 * r, 2 * r] = 1.0
        p["W2"][2 * r + 1, 2 * r + 1] = 1.0
        p["W3"][2 * r, r] = 1.0
        p["W3"][2 * r + 1, r] = -1.0
    g0 = np.random.default_rng(3).standard_normal((Q,) + shape)
    g1 = ob.step_open(lat, g0, "mlp", params=p, limit=False)
    assert np.abs(g1 - ob.step_open(lat, g0, "copy")).max() < 1e-14 * np.abs(g1).max()
    g2 = ob.run_open(lat, g0, 2, "mlp", params=p, limit=False)
    want = ob.step_open(lat, g1, "external", params=ob.ghost_values(lat, g0, "copy"))
    assert np.abs(g2 - want).max() < 1e-14 * np.abs(want).max()
    assert np.abs(g2 - ob.step_open(lat, g1, "copy")).max() > 1e-3 * np.abs(want).max()  # history matters


@pytest.mark.parametrize("name", ["D2Q9", "D2Q5", "D3Q7", "D3Q19", "D1Q3"])
def test_network_closure_never_adds_energy(name):
    """With the energy limit, a network closure cannot raise the weighted energy of the open box
    at tau = 1/2, whatever it predicts: random networks with large biases, random states, every
    step.  Without the limit the same networks do raise it (so the property is not vacuous)."""
    lat = L.get(name)
    shape = {1: (9,), 2: (7, 9), 3: (4, 5, 6)}[lat.D]
    k = len(ob.incoming_canonical(lat))
    grew_without = False
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        p = mlp.init_params(rng, 6 * lat.Q, k)
        p["b1"] = rng.standard_normal(64)
        p["b3"] = 3.0 * rng.standard_normal(k)
        g = rng.standard_normal((lat.Q,) + shape) * lat.fstar.reshape((-1,) + (1,) * lat.D)
        e0 = lbe.weighted_energy(lat, g)
        h = g
        for _ in range(6):
            h2 = ob.step_open(lat, h, "mlp", params=p)
            assert lbe.weighted_energy(lat, h2) <= lbe.weighted_energy(lat, h) * (1 + 1e-12)
            h = h2
        grew_without |= lbe.weighted_energy(lat, ob.step_open(lat, g, "mlp", params=p, limit=False)) > e0
    assert grew_without


@pytest.mark.parametrize("name", ["D2Q9", "D3Q7"])
def test_network_behind_a_sponge_layer(name):
    """The network closure with a sponge layer (width W >= 1).  A network that predicts nothing
    (every weight zero) behind the layer is the sponge closure, bit for bit, over several steps;
    with sigma 0 the layer changes nothing; with damping, a step of any network ends with no more
    weighted energy than the same step without the layer, and with less whenever the layer holds
    a wave."""
    lat = L.get(name)
    shape = {2: (11, 12), 3: (7, 8, 9)}[lat.D]
    k = len(ob.incoming_canonical(lat))
    rng = np.random.default_rng(41)
    g = rng.standard_normal((lat.Q,) + shape) * lat.fstar.reshape((-1,) + (1,) * lat.D)
    nothing = {n: np.zeros_like(v) for n, v in mlp.init_params(rng, 6 * lat.Q, k).items()}
    a = ob.run_open(lat, g, 3, "mlp", params=nothing, sponge_width=3, sponge_sigma=0.4)
    b = ob.run_open(lat, g, 3, "sponge", sponge_width=3, sponge_sigma=0.4)
    assert np.array_equal(a, b)
    p = mlp.init_params(rng, 6 * lat.Q, k)
    p["b3"] = 0.1 * rng.standard_normal(k)
    a = ob.run_open(lat, g, 3, "mlp", params=p, sponge_width=3, sponge_sigma=0.0)
    b = ob.run_open(lat, g, 3, "mlp", params=p)
    assert np.array_equal(a, b)
    h = g
    for _ in range(4):
        damped = ob.step_open(lat, h, "mlp", params=p, sponge_width=3, sponge_sigma=0.4)
        free = ob.step_open(lat, h, "mlp", params=p)
        assert lbe.weighted_energy(lat, damped) < lbe.weighted_energy(lat, free)
        assert not np.array_equal(damped, free)
        h = damped


def test_energy_limit_budget_by_face_count():
    """The limit scales a prediction to E_out / (2^n - 1) only when it exceeds that budget."""
    lat = L.get("D2Q9")
    jin = ob.incoming_canonical(lat)
    jout = np.where(lat.c[:, 0] == -1)[0]
    x = np.zeros(3 * lat.Q)
    x[jout] = [1.0, 2.0, -1.0]
    e_out = float(np.sum(x[jout] ** 2 / lat.fstar[jout]))
    y = np.array([3.0, -1.0, 0.5])
    e_in = float(np.sum(y ** 2 / lat.fstar[jin]))
    for n in (1, 2, 3):
        got = ob.energy_limit(lat, x, y, n)
        budget = e_out / (2 ** n - 1)
        if e_in > budget:
            assert abs(float(np.sum(got ** 2 / lat.fstar[jin])) - budget) < 1e-12 * budget
            assert np.allclose(got / y, got[0] / y[0])
        else:
            assert np.array_equal(got, y)
    small = y * 1e-3
    assert np.array_equal(ob.energy_limit(lat, x, small, 1), small)


def test_face_frames_are_lattice_symmetries():
    for name in ("D2Q9", "D3Q19", "D3Q7", "D2Q5"):
        lat = L.get(name)
        for a, side in ob.faces(lat.D):
            M = ob.face_transform(a, side)
            n_out = np.zeros(3, dtype=np.int64)
            n_out[a] = -1 if side == 0 else 1
            assert np.array_equal(M @ n_out, [-1, 0, 0])
            perm = ob.canonical_perm(lat, a, side)
            assert sorted(perm) == list(range(lat.Q))
            assert np.allclose(lat.fstar[perm], lat.fstar)
            # the canonical entering set is the face's entering set: c . n_out < 0
            jin = ob.incoming_canonical(lat)
            assert set(perm[jin]) == set(np.where(lat.c @ n_out < 0)[0])


def _flip_equivariant_network(lat, rng):
    """A width-64 network f(x) = g(x) + rho g(pi x) built from a random width-32 network g,
    where pi reflects the tangential axis in the canonical frame (c'_y -> -c'_y) on the strip
    and rho is the same reflection on the entering populations: f(pi x) = rho f(x) exactly."""
    Q = lat.Q
    jin = ob.incoming_canonical(lat)
    k = len(jin)
    refl = np.array([np.where((lat.c == lat.c[j] * np.array([1, -1, 1])).all(axis=1))[0][0] for j in range(Q)])
    pi = np.concatenate([m * Q + refl for m in range(6)])  # (pi x)[n] = x[pi[n]], both time levels
    rho = np.array([list(jin).index(refl[j]) for j in jin])
    g = mlp.init_params(rng, 6 * Q, k, hidden=32)
    g["b1"] = 0.1 * rng.standard_normal(32)
    g["b2"] = 0.1 * rng.standard_normal(32)
    g["b3"] = 0.1 * rng.standard_normal(k)
    W1b = np.zeros_like(g["W1"])
    W1b[pi] = g["W1"]  # (pi z) . W1 = z . W1b
    p = {"W1": np.hstack([g["W1"], W1b]), "b1": np.concatenate([g["b1"], g["b1"]]),
         "W2": np.block([[g["W2"], np.zeros((32, 32))], [np.zeros((32, 32)), g["W2"]]]),
         "b2": np.concatenate([g["b2"], g["b2"]]),
         "W3": np.vstack([g["W3"], g["W3"][:, rho]]), "b3": g["b3"] + g["b3"][rho]}
    return p, pi, rho


def test_flip_equivariant_network_construction():
    lat = L.get("D2Q9")
    rng = np.random.default_rng(5)
    p, pi, rho = _flip_equivariant_network(lat, rng)
    x = rng.standard_normal((10, 54))
    assert np.allclose(mlp.predict(p, x[:, pi]), mlp.predict(p, x)[:, rho], atol=1e-14)


def test_network_closure_respects_square_symmetry():
    """A symmetric state in a square box: with a flip-equivariant network every face sees the
    same strips in its own frame, so the open step keeps all eight symmetries of the square.
    With a generic network only the main-diagonal reflection (which maps every face frame onto
    another face frame without a tangential flip) holds."""
    lat = L.get("D2Q9")
    n = 12
    p0 = inputs.gaussian_pressure((n, n), [inputs.Pulse((n / 2 - 0.5, n / 2 - 0.5), 1e-3, 2.5)])
    g = lbe.equilibrium(lat, *inputs.fields_from_pressure(p0, lat.rho0, lat.theta0, lat.gamma))
    params, _, _ = _flip_equivariant_network(lat, np.random.default_rng(4))
    p = lbe.moments(lat, ob.run_open(lat, g, 8, "mlp", params=params))["p"]
    scale = np.abs(p).max()
    for img in (p.T, p[::-1, :], p[:, ::-1], p[::-1, ::-1], p.T[::-1, :]):
        assert np.abs(p - img).max() < 1e-12 * scale
    generic = mlp.init_params(np.random.default_rng(6), 54, 3)
    p = lbe.moments(lat, ob.run_open(lat, g, 8, "mlp", params=generic))["p"]
    assert np.abs(p - p.T).max() < 1e-12 * np.abs(p).max()


def test_mlp_gradients_match_finite_differences():
    rng = np.random.default_rng(7)
    p = mlp.init_params(rng, 27, 3)
    for key in p:
        if key.startswith("b"):
            p[key] = 0.1 * rng.standard_normal(p[key].shape)
    x = rng.standard_normal((40, 27))
    t = rng.standard_normal((40, 3))
    z, _ = mlp.normalise(x)
    y, cache = mlp.forward(p, z)
    g = mlp.backward(p, cache, y, t)
    h = 1e-6
    for key in p:
        flat_idx = rng.choice(p[key].size, size=min(6, p[key].size), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, p[key].shape)
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[key][idx] += h
            pm[key][idx] -= h
            fd = (mlp.mse(mlp.forward(pp, z)[0], t) - mlp.mse(mlp.forward(pm, z)[0], t)) / (2 * h)
            assert abs(fd - g[key][idx]) < 1e-6 * max(1.0, abs(fd)), (key, idx, fd, g[key][idx])


def test_quantized_gradients_are_close_to_exact():
    rng = np.random.default_rng(8)
    p = mlp.init_params(rng, 21, 1)
    x = rng.standard_normal((256, 21))
    t = rng.standard_normal((256, 1))
    z, _ = mlp.normalise(x)
    y, c = mlp.forward(p, z)
    yq, cq = mlp.forward(p, z, quantize=True)
    g = mlp.backward(p, c, y, t)
    gq = mlp.backward(p, cq, yq, t, quantize=True)
    for key in p:
        # bf16 keeps 8 significant bits at every GEMM input: a few per cent after three layers
        assert np.linalg.norm(gq[key] - g[key]) <= 5e-2 * np.linalg.norm(g[key]), key


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5e-3, 0.0])
    got = mlp.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3*2^-8 ties up to 1 + 2^-6
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -6 and got[3] == 1.0
    assert abs(got[4] - vals[4]) <= 2 ** -9 * abs(vals[4]) and got[5] == 0.0


def test_adam_first_step_is_signed_learning_rate():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 0.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    mlp.adam(p, g, m, v, 1, lr=0.01, eps=1e-12)
    assert np.allclose(p["w"], [0.99, -1.99, 3.0], atol=1e-9)


def test_adam_bias_correction_over_many_steps():
    """With a constant gradient g the bias-corrected moments are exactly m_hat = g and
    v_hat = g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so every step moves a
    parameter by lr g / (|g| + eps).  A bias correction with any other exponent than t fails this
    from t = 2 on (at t = 1 every exponent agrees)."""
    g0 = np.array([0.5, -1e-3, 2.0, -7.0])
    p = {"w": np.array([1.0, -2.0, 3.0, 0.25])}
    g = {"w": g0.copy()}
    m = {"w": np.zeros(4)}
    v = {"w": np.zeros(4)}
    lr, eps = 0.01, 1e-12
    for t in range(1, 11):
        before = p["w"].copy()
        mlp.adam(p, g, m, v, t, lr=lr, b1=0.9, b2=0.999, eps=eps)
        assert np.allclose(before - p["w"], lr * g0 / (np.abs(g0) + eps), rtol=1e-12, atol=0), t
        assert np.allclose(m["w"], (1 - 0.9 ** t) * g0, rtol=1e-13, atol=0), t
        assert np.allclose(v["w"], (1 - 0.999 ** t) * g0 ** 2, rtol=1e-12, atol=0), t


def test_adam_planted_bias_correction_mistake_is_caught():
    """The pin above is not vacuous: the same loop with the bias correction frozen at t = 1
    (a wrong exponent) departs from lr g / |g| at t = 2."""
    g0 = np.array([0.5, -2.0])
    m, v = np.zeros(2), np.zeros(2)
    steps = []
    for t in range(1, 3):
        m = 0.9 * m + 0.1 * g0
        v = 0.999 * v + 0.001 * g0 ** 2
        mh, vh = m / (1 - 0.9 ** 1), v / (1 - 0.999 ** 1)  # planted: exponent 1 instead of t
        steps.append(0.01 * mh / (np.sqrt(vh) + 1e-12))
    assert np.allclose(steps[0], 0.01 * np.sign(g0))
    assert not np.allclose(steps[1], 0.01 * np.sign(g0), rtol=1e-6)


def test_normalise_scale_is_the_root_mean_square():
    """s is the root mean square of each row, from hand-computable rows: [3, 4, 0, ...] of length n
    has s = 5 / sqrt(n) (its mean |x| is 7 / n, so a mean in place of the RMS fails); a constant
    row c has s = |c|; a row scaled by 2^-120 (squares below FP64's normal range) has its s scaled
    exactly by 2^-120; an all-zero row has s = 0 and z = 0; z = x / s in every other row."""
    n = 21
    rows = np.zeros((5, n))
    rows[0, :2] = [3.0, 4.0]
    rows[1, :] = -0.75
    rows[2, :2] = [3.0 * 2.0 ** -120, 4.0 * 2.0 ** -120]
    rows[3, :] = np.arange(1, n + 1, dtype=np.float64)
    z, s = mlp.normalise(rows)
    s = s.ravel()
    want = [5.0 / np.sqrt(n), 0.75, 5.0 / np.sqrt(n) * 2.0 ** -120,
            np.sqrt(np.sum(np.arange(1, n + 1) ** 2.0) / n), 0.0]
    for k in range(5):
        assert abs(s[k] - want[k]) <= 1e-15 * want[k], k
    assert s[0] != 7.0 / n
    assert np.all(z[4] == 0.0)
    for k in range(4):
        assert np.allclose(z[k] * s[k], rows[k], rtol=1e-15, atol=0)
        assert abs(np.sqrt(np.mean(z[k] ** 2)) - 1.0) <= 1e-15


def test_flat_layout_roundtrip():
    p = mlp.init_params(np.random.default_rng(0), 27, 3)
    v = mlp.flat(p)
    assert v.size == 27 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    q = mlp.unflat(v, 27, 3)
    assert all(np.array_equal(p[k], q[k]) for k in p)
