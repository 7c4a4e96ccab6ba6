"""The Langevin O-step of Algorithm 1 on the GPU against the oracle driven by the same
noise: both sides implement the counter-based generator (Philox4x32-10) and the
Box-Muller map from their published definitions, so the k-th O-step gives atom i the same
normals.  Also: the single-time-step form, the exact-list fallback reusing its noise,
bitwise resume across calls, the bath temperature, and argument checks."""

import numpy as np
import pytest
import torch

from _gpu_common import OI, OP, oracle_model, say, system, weights, SPECS
from oracle.rng import OStepNoise
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu

GAMMA, TEMP, SEED = 0.02, 300.0, 4242


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _state(sy, dt, n_inner, thermo=True):
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128)
    if thermo:
        st.set_thermostat(GAMMA, TEMP, SEED)
    return st


def _oracle_force(which, sy):
    m = oracle_model(which)

    def f(x):
        E, F, _ = OP.energy_forces(m, x, sy.species, sy.box)
        return E[0], F
    return f


def test_langevin_dmts_matches_oracle_water192(models):
    say("Langevin DMTS water192 3 outer x (4 inner), dt 2 fs")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    st = _state(sy, 2.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, models["small"], models["large"], 3)
    assert st.o_steps == 12
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    noise = OStepNoise(o.m, GAMMA, TEMP, SEED)
    fs, fl = _oracle_force("small", sy), _oracle_force("large", sy)
    for _ in range(3):
        OI.mts_step(o, 2.0, 4, fs, fl, thermo=noise)
    assert noise.k == 12
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    assert np.max(np.abs(api.from_soa(v) - o.v)) < 1e-8
    # the noise is not negligible: the NVE trajectory is far from this one
    o2 = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    for _ in range(3):
        OI.mts_step(o2, 2.0, 4, fs, fl)
    assert np.max(np.abs(o2.v - o.v)) > 1e-4


def test_langevin_single_time_step_matches_oracle(models):
    say("Langevin BAOAB water192 10 x 0.5 fs")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    st = _state(sy, 0.5, 1)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, None, models["small"], 10)
    assert st.o_steps == 10
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    noise = OStepNoise(o.m, GAMMA, TEMP, SEED)
    f = _oracle_force("small", sy)
    for _ in range(10):
        OI.sts_step(o, 0.5, f, thermo=noise)
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    assert np.max(np.abs(api.from_soa(v) - o.v)) < 1e-8


def test_langevin_fallback_reuses_its_noise(models):
    """A call redone with exact lists draws the same O-step numbers again."""
    say("Langevin shared-list fallback")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    v0[7] = [0.35, 0.0, 0.0]
    st = _state(sy, 4.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, models["small"], models["large"], 1)
    assert st.fallbacks == 1 and st.o_steps == 4
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    OI.mts_step(o, 4.0, 4, _oracle_force("small", sy), _oracle_force("large", sy),
                thermo=OStepNoise(o.m, GAMMA, TEMP, SEED))
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    assert np.max(np.abs(api.from_soa(v) - o.v)) < 1e-8


def test_langevin_resume_and_seed(models):
    """Two calls continue the noise of one call bit for bit; another seed gives another
    trajectory; set_thermostat restarts the counter."""
    say("Langevin resume / seed")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a = _state(sy, 4.0, 4)
    xa, va = api.to_soa(sy.pos), api.to_soa(v0)
    a.step(xa, va, models["small"], models["large"], 4)
    b = _state(sy, 4.0, 4)
    xb, vb = api.to_soa(sy.pos), api.to_soa(v0)
    b.step(xb, vb, models["small"], models["large"], 2)
    b.step(xb, vb, models["small"], models["large"], 2)
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert a.o_steps == b.o_steps == 16
    c = _state(sy, 4.0, 4)
    c.set_thermostat(GAMMA, TEMP, SEED + 1)
    xc, vc = api.to_soa(sy.pos), api.to_soa(v0)
    c.step(xc, vc, models["small"], models["large"], 4)
    assert not torch.equal(vc, va)
    b.set_thermostat(GAMMA, TEMP, SEED)
    assert b.o_steps == 0


def test_thermostat_reaches_bath_temperature_water4500(models):
    """From rest, strong friction brings the 4,500-atom box to the bath temperature: the
    mean kinetic temperature (3N degrees of freedom, all thermostatted) over the second
    half of 60 outer steps is within 3% of 300 K, and the velocities of the last step
    follow the Maxwell-Boltzmann distribution of each species (Kolmogorov-Smirnov)."""
    say("Langevin water4500 bath temperature")
    sy = system("water4500")
    st = _state(sy, 4.0, 4, thermo=False)
    st.set_thermostat(0.05, TEMP, 99)
    x = api.to_soa(sy.pos)
    v = torch.zeros_like(x)
    temps = []
    for k in range(60):
        e = st.step(x, v, models["small"], models["large"], 1)
        if k >= 30:
            temps.append(2.0 * e[2].item() / (3 * sy.n_atoms * OI.K_BOLTZMANN))
    say(f"mean T {np.mean(temps):.1f} K")
    assert abs(np.mean(temps) / TEMP - 1.0) < 0.03
    # Maxwell-Boltzmann: each velocity component, scaled by sqrt(m / (k_B T KAPPA)), is a
    # standard normal; Kolmogorov-Smirnov over the 13,500 components of the last step,
    # hydrogen and oxygen separately (the scale depends on the mass)
    from scipy import stats
    vv = v.cpu().numpy()
    m = synth.MASSES[sy.species]
    z = vv * np.sqrt(m / (OI.K_BOLTZMANN * TEMP * OI.KAPPA))[None, :]
    for sp_id in np.unique(sy.species):
        sample = z[:, sy.species == sp_id].ravel()
        ks = stats.kstest(sample, "norm")
        say(f"species {sp_id}: {sample.size} components, KS D {ks.statistic:.4f}, p {ks.pvalue:.3f}")
        assert ks.pvalue > 1e-3


def test_thermostat_rejects_bad_arguments():
    sy = system("water192")
    st = _state(sy, 2.0, 4, thermo=False)
    for g, t in [(-1e-3, 300.0), (float("nan"), 300.0), (1e-3, -1.0), (1e-3, float("inf"))]:
        with pytest.raises(api.DmtsError) as e:
            st.set_thermostat(g, t, 1)
        assert e.value.status == api.E_ARG
