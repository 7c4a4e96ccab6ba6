"""The oracle's counter-based generator and Langevin O-step against what the generator's
publication and the mathematics fix: known-answer vectors, the normal distribution of the
Box-Muller deviates, the invariance of the Maxwell-Boltzmann distribution under the exact
Ornstein-Uhlenbeck update, and the kinetic temperature of thermostatted dynamics."""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import integrators as OI
from oracle.rng import OStepNoise, o_step_normals, philox4x32_10

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(w, 16) for w in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(np.array([r[0:4]], dtype=np.uint64), np.array([r[4:6]], dtype=np.uint64))
        assert [int(x) for x in out[0]] == r[6:10]


def test_philox_planted_mistakes_fail_the_known_answers():
    """A wrong multiplier or a missing key bump changes every known answer."""
    r = _kat()[2]
    ctr, key = np.array([r[0:4]], dtype=np.uint64), np.array([r[4:6]], dtype=np.uint64)
    good = [int(x) for x in philox4x32_10(ctr, key)[0]]
    import oracle.rng as R
    saved = R.W0
    try:
        R.W0 = np.uint64(0)
        assert [int(x) for x in philox4x32_10(ctr, key)[0]] != good
    finally:
        R.W0 = saved


def test_normals_are_standard_normal():
    xi = np.concatenate([o_step_normals(20000, k, seed=12345) for k in range(5)])  # 300k
    flat = xi.ravel()
    n = flat.size
    assert abs(flat.mean()) < 5.0 / np.sqrt(n)
    assert abs(flat.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    for d in range(3):
        assert stats.kstest(xi[:, d], "norm").pvalue > 1e-4
    c = np.corrcoef(xi.T)
    assert np.max(np.abs(c - np.eye(3))) < 5.0 / np.sqrt(xi.shape[0])


def test_streams_differ_by_atom_step_and_seed():
    a = o_step_normals(1000, 7, seed=1)
    assert np.array_equal(a, o_step_normals(1000, 7, seed=1))
    assert not np.any(a == o_step_normals(1000, 8, seed=1))
    assert not np.any(a == o_step_normals(1000, 7, seed=2))
    assert len(np.unique(a[:, 0])) == 1000
    # the step counter's high word enters the counter
    assert not np.any(o_step_normals(10, 5, 3) == o_step_normals(10, 5 + (1 << 32), 3))


def test_o_step_keeps_maxwell_boltzmann():
    """If v ~ MB(T), c v + sqrt((1 - c^2) k_B T KAPPA / m) xi ~ MB(T) for any c."""
    rng = np.random.default_rng(5)
    n, T = 40000, 300.0
    m = rng.choice([1.008, 15.999], size=n)
    sd = np.sqrt(OI.K_BOLTZMANN * T * OI.KAPPA / m)
    v = rng.standard_normal((n, 3)) * sd[:, None]
    noise = OStepNoise(m, gamma=0.3, T=T, seed=9)
    for _ in range(3):
        v = noise(v, 1.0)
    z = v / sd[:, None]
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-4


def test_o_step_limits():
    rng = np.random.default_rng(2)
    m = np.full(50, 12.0)
    v = rng.standard_normal((50, 3))
    assert np.array_equal(OI.langevin_o(v, m, 1.0, 0.0, 300.0, np.ones((50, 3))), v)
    xi = o_step_normals(50, 0, 4)
    full = OI.langevin_o(v, m, 1.0, 1e3, 300.0, xi)   # c = 0: a fresh MB sample
    np.testing.assert_allclose(full, np.sqrt(OI.K_BOLTZMANN * 300.0 * OI.KAPPA / 12.0) * xi,
                               rtol=1e-14)


def test_thermostatted_respa_reaches_the_bath_temperature():
    """Algorithm 1 with the O-step on independent 3-D harmonic oscillators (fast part a
    stiff spring, slow part a soft one): the mean kinetic temperature of the second half
    of the run is the bath temperature."""
    n, T = 3000, 300.0
    rng = np.random.default_rng(8)
    m = np.full(n, 16.0)
    k_fast, k_slow = 2.0, 0.5   # eV / A^2

    def fast(x):
        return 0.5 * k_fast * np.sum(x * x), -k_fast * x

    def full(x):
        return 0.5 * (k_fast + k_slow) * np.sum(x * x), -(k_fast + k_slow) * x

    st = OI.MTSState(x=0.05 * rng.standard_normal((n, 3)), v=np.zeros((n, 3)), m=m)
    noise = OStepNoise(m, gamma=0.05, T=T, seed=77)
    temps = []
    for step in range(400):
        OI.mts_step(st, 2.0, 2, fast, full, thermo=noise)
        if step >= 200:
            temps.append(2.0 * OI.kinetic_energy(st.v, m) / (3 * n * OI.K_BOLTZMANN))
    assert noise.k == 800
    assert abs(np.mean(temps) / T - 1.0) < 0.02
