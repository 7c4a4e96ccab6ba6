"""Pins of the oracle's integrators (Algorithm 1 and the single-time-step baseline)
against closed forms and exact properties: the harmonic oscillator's discrete phase
advance under velocity Verlet, the linear transfer matrix of one RESPA step, exact
reduction of Algorithm 1 to velocity Verlet when both levels are the same model, time
reversibility, second-order energy error, and the Ornstein-Uhlenbeck O-step moments."""

import math

import numpy as np
import pytest

from oracle import integrators as I
from oracle import potentials as P
from paper_2510_06562_amd import synth


def _harmonic(k):
    def f(x):
        return 0.5 * k * float(np.sum(x * x)), -k * x
    return f


def test_kappa_value():
    # 1 eV/(A amu) = 9.6485332e-3 A/fs^2 (e/u = 9.6485332e7 C/kg, CODATA)
    assert I.KAPPA == pytest.approx(9.648533215665e-3, rel=1e-12)


def test_verlet_phase_advance_harmonic():
    """For x'' = -w^2 x, velocity Verlet advances the phase by theta per step with
    cos(theta) = 1 - (w dt)^2 / 2 (a textbook property of the Stormer-Verlet map)."""
    k, m, dt = 2.0, np.array([3.0]), 0.7
    w = math.sqrt(k * I.KAPPA / m[0])
    st = I.MTSState(x=np.array([[1.0, 0, 0]]), v=np.zeros((1, 3)), m=m)
    xs = [st.x[0, 0]]
    for _ in range(200):
        I.sts_step(st, dt, _harmonic(k))
        xs.append(st.x[0, 0])
    theta = math.acos(1 - (w * dt) ** 2 / 2)
    # starting at rest at x = 1, the exact discrete solution is x_n = A cos(n theta) + B sin
    # with x_0 = 1 and x_1 = 1 - (w dt)^2 / 2 => x_n = cos(n theta)
    np.testing.assert_allclose(xs, np.cos(theta * np.arange(201)), atol=1e-12)


def _kick_mat(tau, k, m):
    return np.array([[1.0, 0.0], [-tau * I.KAPPA * k / m, 1.0]])


def _drift_mat(tau):
    return np.array([[1.0, tau], [0.0, 1.0]])


@pytest.mark.parametrize("n_slow", [1, 3, 4])
def test_respa_step_is_the_transfer_matrix_product(n_slow):
    """With linear forces F_small = -k_s x and F = -k_L x every sub-step is a 2x2 matrix on
    (x, v); one outer step must equal their product."""
    ks, kL, m, dt = 5.0, 4.2, 2.0, 1.3
    h = dt / n_slow
    inner = _kick_mat(h / 2, ks, m) @ _drift_mat(h / 2) @ _drift_mat(h / 2) @ _kick_mat(h / 2, ks, m)
    T = _kick_mat(dt / 2, kL - ks, m) @ np.linalg.matrix_power(inner, n_slow) @ _kick_mat(dt / 2, kL - ks, m)
    x0, v0 = 0.8, -0.05
    st = I.MTSState(x=np.array([[x0, 0, 0]]), v=np.array([[v0, 0, 0]]), m=np.array([m]))
    for _ in range(5):
        I.mts_step(st, dt, n_slow, _harmonic(ks), _harmonic(kL))
    exp = np.linalg.matrix_power(T, 5) @ np.array([x0, v0])
    np.testing.assert_allclose([st.x[0, 0], st.v[0, 0]], exp, rtol=1e-13, atol=1e-15)
    assert np.linalg.det(T) == pytest.approx(1.0, abs=1e-13)   # symplectic in 1D


@pytest.mark.parametrize("n_slow", [1, 4])
def test_monitored_step_follows_the_transfer_matrices(n_slow):
    """The force-difference guard on a 1-d oscillator with F_small = -k_s x and
    F = -k_L x: below the threshold the step is the RESPA matrix product; above it the
    step is n_slow velocity-Verlet steps of dt/n_slow with k_L, and the recorded breach is
    |k_L - k_s| max(|x_0|, |x_1|), x_1 the end of the discarded RESPA step."""
    ks, kL, m, dt = 5.0, 4.2, 2.0, 1.3
    h = dt / n_slow
    inner = _kick_mat(h / 2, ks, m) @ _drift_mat(h / 2) @ _drift_mat(h / 2) @ _kick_mat(h / 2, ks, m)
    T = _kick_mat(dt / 2, kL - ks, m) @ np.linalg.matrix_power(inner, n_slow) @ _kick_mat(dt / 2, kL - ks, m)
    V = np.linalg.matrix_power(_kick_mat(h / 2, kL, m) @ _drift_mat(h) @ _kick_mat(h / 2, kL, m), n_slow)
    x0, v0 = 0.8, -0.05
    x1 = (T @ np.array([x0, v0]))[0]
    breach = abs(kL - ks) * max(abs(x0), abs(x1))

    def run(thr):
        st = I.MTSState(x=np.array([[x0, 0, 0]]), v=np.array([[v0, 0, 0]]), m=np.array([m]))
        return I.mts_step_monitored(st, dt, n_slow, _harmonic(ks), _harmonic(kL), thr)

    kept, b, redo = run(breach * (1 + 1e-9))
    assert not redo and b == pytest.approx(breach, rel=1e-14)
    np.testing.assert_allclose([kept.x[0, 0], kept.v[0, 0]], T @ [x0, v0], rtol=1e-13)
    redone, b, redo = run(breach * (1 - 1e-9))
    assert redo and b == pytest.approx(breach, rel=1e-14)
    np.testing.assert_allclose([redone.x[0, 0], redone.v[0, 0]], V @ [x0, v0], rtol=1e-13)
    assert redone.first_step


SMALL = P.make_model(0, 3.5, 16, 64, synth.model_weights(synth.SMALL, synth.SMALL_SEED),
                     energy_scale=1.0)


def _force(model, box):
    def f(x):
        E, F, _ = P.energy_forces(model, x, _force.sp, box)
        return E[0], F
    return f


def test_respa_reduces_exactly_to_verlet_when_levels_coincide():
    """F - F_small == 0 exactly when both levels are the same model, so n_slow inner
    steps of dt/n_slow are bitwise n_slow velocity-Verlet steps."""
    sy = synth.water_192()
    _force.sp = sy.species
    f = _force(SMALL, sy.box)
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a = I.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    b = I.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    for _ in range(2):
        I.mts_step(a, 2.0, 4, f, f)
    for _ in range(8):
        I.sts_step(b, 0.5, f)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)


def test_time_reversibility():
    """k steps forward, v -> -v, k steps back returns to the start (the RESPA property the
    method relies on)."""
    pos = synth.water_192().pos[:45]
    sp = synth.water_192().species[:45]
    _force.sp = sp
    large = P.make_model(1, 5.2, 32, 128, synth.model_weights(synth.LARGE, synth.LARGE_SEED),
                         energy_scale=1.0)
    fs = _force(SMALL, 0.0)
    fl = _force(large, 0.0)
    st = I.MTSState(x=pos.copy(), v=synth.maxwell_boltzmann(sp, 300.0, 1), m=synth.MASSES[sp])
    for _ in range(6):
        I.mts_step(st, 2.0, 4, fs, fl)
    st.v = -st.v
    for _ in range(6):
        I.mts_step(st, 2.0, 4, fs, fl)
    assert np.max(np.abs(st.x - pos)) < 1e-10


def test_energy_error_is_second_order():
    """Max |H(t) - H(0)| of velocity Verlet over a fixed time scales as dt^2."""
    sy = synth.water_192()
    pos, sp = sy.pos[:60], sy.species[:60]
    _force.sp = sp
    f = _force(SMALL, 0.0)
    v0 = synth.maxwell_boltzmann(sp, 300.0, 3)
    devs = []
    for dt in (0.4, 0.2):
        st = I.MTSState(x=pos.copy(), v=v0.copy(), m=synth.MASSES[sp])
        I.sts_step(st, 0.0, f)
        H0 = I.conserved_energy(st)
        dev = 0.0
        for _ in range(int(round(8.0 / dt))):
            I.sts_step(st, dt, f)
            dev = max(dev, abs(I.conserved_energy(st) - H0))
        devs.append(dev)
    assert 3.0 < devs[0] / devs[1] < 5.0


def test_nve_water192_conserves_energy():
    """The 192-atom water run: 20 velocity-Verlet steps of 0.5 fs with the fast model."""
    sy = synth.water_192()
    _force.sp = sy.species
    model = P.make_model(0, 3.5, 16, 64, synth.model_weights(synth.SMALL, synth.SMALL_SEED))
    f = _force(model, sy.box)
    st = I.MTSState(x=sy.pos.copy(), v=synth.maxwell_boltzmann(sy.species, 300.0, 200),
                    m=sy.masses())
    I.sts_step(st, 0.0, f)
    H = [I.conserved_energy(st)]
    for _ in range(20):
        I.sts_step(st, 0.5, f)
        H.append(I.conserved_energy(st))
    H = np.array(H)
    KE = I.kinetic_energy(st.v, st.m)
    assert np.max(np.abs(H - H[0])) < 1e-6 * KE


def test_langevin_o_step_moments():
    """O-step from v = 0: the new velocity is Gaussian with variance (1 - c^2) k_B T / m
    (times KAPPA for A/fs units), c = exp(-gamma h); and from v it decays by c on average."""
    n = 200_000
    m = np.full(n, 16.0)
    rng = np.random.default_rng(0)
    xi = rng.standard_normal((n, 3))
    gamma, h, T = 1e-3, 1.0, 300.0
    v = I.langevin_o(np.zeros((n, 3)), m, h, gamma, T, xi)
    c = math.exp(-gamma * h)
    var = (1 - c * c) * I.K_BOLTZMANN * T * I.KAPPA / 16.0
    assert np.var(v) == pytest.approx(var, rel=0.01)
    v1 = I.langevin_o(np.ones((n, 3)), m, h, gamma, T, xi)
    assert np.mean(v1) == pytest.approx(c, abs=5e-3 * math.sqrt(var) + 1e-12)
    assert np.array_equal(I.langevin_o(v1, m, h, 0.0, T, xi), v1)


def test_maxwell_boltzmann_temperature():
    sy = synth.water_4500()
    v = synth.maxwell_boltzmann(sy.species, 300.0, 201)
    T = I.temperature(v, sy.masses())
    assert abs(T - 300.0) < 12.0          # 3N-3 = 13,497 dof -> sd ~ 3.7 K
    np.testing.assert_allclose((sy.masses()[:, None] * v).sum(0), 0.0, atol=1e-10)
