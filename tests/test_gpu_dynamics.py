"""GPU dynamics through dmts_step against the oracle's integrators, plus the exact
properties the device path must keep on its own: Algorithm 1 collapses bitwise to
velocity Verlet when both levels are the same model, time reversibility, bitwise
resume, and energy conservation."""

import numpy as np
import pytest
import torch

from _gpu_common import OI, OP, oracle_model, say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _state(sy, dt, n_inner):
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    return api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128), sp


def _oracle_force(which, sy):
    m = oracle_model(which)

    def f(x):
        E, F, _ = OP.energy_forces(m, x, sy.species, sy.box)
        return E[0], F
    return f


def test_velocity_verlet_trajectory_water192(models):
    """The 192-atom water run: 20 velocity-Verlet steps of 0.5 fs with the fast model."""
    say("VV water192 20 x 0.5 fs")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    st, _ = _state(sy, 0.5, 1)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    en = st.step(x, v, None, models["small"], 20)
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    f = _oracle_force("small", sy)
    for _ in range(20):
        OI.sts_step(o, 0.5, f)
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    assert np.max(np.abs(api.from_soa(v) - o.v)) < 1e-8
    e = en.cpu().numpy()
    assert e[0] == pytest.approx(o.E, abs=1e-6)
    assert e[2] == pytest.approx(OI.kinetic_energy(o.v, o.m), rel=1e-8)


def test_dmts_matches_oracle_algorithm1_water192(models):
    say("DMTS water192 3 outer x (4 inner), dt 2 fs")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    st, _ = _state(sy, 2.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    en = st.step(x, v, models["small"], models["large"], 3)
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    fs, fl = _oracle_force("small", sy), _oracle_force("large", sy)
    for _ in range(3):
        OI.mts_step(o, 2.0, 4, fs, fl)
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    assert np.max(np.abs(api.from_soa(v) - o.v)) < 1e-8
    e = en.cpu().numpy()
    assert e[0] == pytest.approx(o.E, abs=1e-6) and e[1] == pytest.approx(o.E_small, abs=1e-6)


def test_fast_atom_triggers_exact_fallback(models):
    """An atom fast enough to leave the shared list's skin within one call: the call is
    redone with exact lists and still follows Algorithm 1 of the oracle."""
    say("shared-list fallback")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    v0[7] = [0.35, 0.0, 0.0]          # 1.4 A per 4 fs outer step (skin half-width 0.85 A)
    st, _ = _state(sy, 4.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, models["small"], models["large"], 1)
    assert st.fallbacks == 1
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    OI.mts_step(o, 4.0, 4, _oracle_force("small", sy), _oracle_force("large", sy))
    assert np.max(np.abs(api.from_soa(x) - o.x)) < 1e-7
    # a normal call afterwards stays on the shared list
    v[:, 7] = 0.0
    st.step(x, v, models["small"], models["large"], 1)
    assert st.fallbacks == 1


def test_respa_collapses_bitwise_to_verlet(models):
    """F - F_small is exactly zero when both levels are one model, so Algorithm 1 with
    n inner steps is n velocity-Verlet steps of dt/n, bit for bit."""
    say("RESPA -> VV bitwise")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    m = models["small"]
    a, _ = _state(sy, 2.0, 4)
    b, _ = _state(sy, 0.5, 1)
    xa, va = api.to_soa(sy.pos), api.to_soa(v0)
    xb, vb = api.to_soa(sy.pos), api.to_soa(v0)
    a.step(xa, va, m, m, 3)
    b.step(xb, vb, None, m, 12)
    assert torch.equal(xa, xb) and torch.equal(va, vb)


def test_time_reversibility(models):
    say("reversibility")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    st, _ = _state(sy, 3.0, 3)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, models["small"], models["large"], 10)
    v.neg_()
    st.step(x, v, models["small"], models["large"], 10)
    assert np.max(np.abs(api.from_soa(x) - sy.pos)) < 1e-8
    assert np.max(np.abs(api.from_soa(v) + v0)) < 1e-9


def test_resume_is_bitwise(models):
    """Restarting from saved (x, v) recomputes both forces on the first step and continues
    exactly as an uninterrupted run."""
    say("resume")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a, _ = _state(sy, 4.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    a.step(x, v, models["small"], models["large"], 2)
    xs, vs = x.clone(), v.clone()
    a.step(x, v, models["small"], models["large"], 3)
    b, _ = _state(sy, 4.0, 4)
    b.step(xs, vs, models["small"], models["large"], 3)
    assert torch.equal(x, xs) and torch.equal(v, vs)


def test_dmts_energy_conservation_water4500(models):
    """Short NVE run of the 4,500-atom box (DMTS 1 fs / 4 fs): the conserved energy
    KE + E_large wanders by far less than kT per atom."""
    say("NVE water4500 DMTS 100 outer steps")
    sy = system("water4500")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 201)
    st, _ = _state(sy, 4.0, 4)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    H = []
    for _ in range(10):
        H.append(st.step(x, v, models["small"], models["large"], 10)[3].item())
    H = np.array(H)
    assert np.max(np.abs(H - H[0])) / sy.n_atoms < 1e-5


def test_state_reports_overflow(models):
    say("state overflow")
    sy = system("water192")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, 1.0, 1, 2, 2)
    x, v = api.to_soa(sy.pos), api.to_soa(np.zeros((sy.n_atoms, 3)))
    with pytest.raises(api.DmtsError) as e:
        st.step(x, v, models["small"], models["large"], 1)
    assert e.value.status == api.E_CAPACITY


def test_state_reports_nonfinite(models):
    say("state nonfinite")
    sy = system("water192")
    st, _ = _state(sy, 1.0, 1)
    pos = sy.pos.copy()
    v0 = np.zeros((sy.n_atoms, 3))
    v0[5, 1] = np.inf
    x, v = api.to_soa(pos), api.to_soa(v0)
    with pytest.raises(api.DmtsError) as e:
        st.step(x, v, None, models["small"], 1)
    assert e.value.status == api.E_NONFINITE
