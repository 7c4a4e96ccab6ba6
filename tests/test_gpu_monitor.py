"""The force-difference monitor: an outer step whose slow kicks see an atom with
|F - F_small| above the threshold is rolled back and redone as single-time-step steps of
the inner length with the reference model (the paper's temporary reversion to STS
integration, Results: protein-ligand complexes).  Checked against the oracle's monitored
step at the paper's threshold (150 kcal/mol/A = 6.505 eV/A), with the breach forced from
the host by moving one atom toward a neighbour; and, device against device, with thresholds
that every step or no step breaches."""

import numpy as np
import pytest
import torch

from _gpu_common import OI, ON, OP, say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu

THRESHOLD = 6.505          # 150 kcal/mol/A in eV/A
STIFF = 4.366              # energy scale of both models: the undisplaced box stays ~6 %
#                            below the threshold, the displaced atom ~6 % above it


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _state(sy, dt, n_inner):
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    return api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128), sp


def _displaced_water():
    """water192 with atom 0 moved 80 % of the way toward its fifth-nearest neighbour."""
    sy = system("water192")
    i, j, d = ON.pairs(sy.pos, sy.box, 3.5, None)
    sel = i == 0
    k = np.argsort(np.linalg.norm(d[sel], axis=1))[4]
    pos = sy.pos.copy()
    pos[0] += 0.8 * d[sel][k]
    return synth.System(pos=pos, species=sy.species, box=sy.box, name="water192-displaced")


def test_breach_at_the_papers_threshold_matches_the_oracle():
    """Three outer steps of 2 fs (four inner steps) from the displaced box: the device
    rolls back and redoes exactly the steps the oracle's monitored step redoes, its
    trajectory matches the oracle's to < 1e-7 A and < 1e-8 A/fs, and the recorded breach
    equals the oracle's largest |F - F_small| of the redone steps to rel. 1e-5."""
    say("monitor: 6.505 eV/A breach vs oracle")
    sy = _displaced_water()
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    ms = OP.make_model(0, 3.5, 16, 64, weights("small"), energy_scale=STIFF)
    ml = OP.make_model(1, 5.2, 32, 128, weights("large"), energy_scale=STIFF)
    fs = lambda x: (lambda r: (r[0][0], r[1]))(OP.energy_forces(ms, x, sy.species, sy.box))  # noqa: E731
    fl = lambda x: (lambda r: (r[0][0], r[1]))(OP.energy_forces(ml, x, sy.species, sy.box))  # noqa: E731
    o = OI.MTSState(x=sy.pos.copy(), v=v0.copy(), m=sy.masses())
    redone, breaches = 0, []
    for _ in range(3):
        o, worst, red = OI.mts_step_monitored(o, 2.0, 4, fs, fl, THRESHOLD)
        # no decision within 1 % of the threshold: FP32 forces cannot flip it
        assert abs(worst - THRESHOLD) > 0.01 * THRESHOLD
        redone += red
        if red:
            breaches.append(worst)
    assert 0 < redone < 3   # some steps reverted, some kept
    small = api.Model.from_spec(SPECS["small"], weights("small"), energy_scale=STIFF)
    large = api.Model.from_spec(SPECS["large"], weights("large"), energy_scale=STIFF)
    st, _ = _state(sy, 2.0, 4)
    st.set_fdiff_threshold(THRESHOLD)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, small, large, 3)
    n, breach = st.fdiff
    say(f"  oracle redid {redone} of 3 steps, breach {max(breaches):.5f}; device {n}, {breach:.5f}")
    assert n == redone
    assert breach == pytest.approx(max(breaches), rel=1e-5)
    # tolerance of the trajectory: these stiff models have forces up to ~8 eV/A, so the
    # FP32 force error (~1e-6 relative, 10x below its 1e-5 bound) moves a hydrogen by
    # KAPPA dF t^2 / (2 m) ~ 0.0096 * 8e-6 * 36 / 2 ~ 1.4e-6 A over the 6 fs and its
    # velocity by KAPPA dF t / m ~ 5e-7 A/fs
    dx = np.max(np.abs(api.from_soa(x) - o.x))
    dv = np.max(np.abs(api.from_soa(v) - o.v))
    say(f"  trajectory: max |dx| {dx:.2e} A, max |dv| {dv:.2e} A/fs")
    assert dx < 2e-6 and dv < 1e-6


@pytest.mark.parametrize("thermo", [False, True])
def test_every_step_breaching_is_single_time_stepping(models, thermo):
    """With a threshold below every force difference each outer step is redone, and the
    trajectory is bit for bit that of single-time-step steps of dt/n with the reference
    model (and the same thermostat noise)."""
    say(f"monitor: breach -> STS (thermostat {thermo})")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a, sp = _state(sy, 2.0, 4)
    b, _ = _state(sy, 0.5, 1)
    if thermo:
        a.set_thermostat(0.02, 300.0, 7)
        b.set_thermostat(0.02, 300.0, 7)
    a.set_fdiff_threshold(1e-9)
    xa, va = api.to_soa(sy.pos), api.to_soa(v0)
    xb, vb = api.to_soa(sy.pos), api.to_soa(v0)
    # the largest |F - F_small| at the start bounds the recorded breach from below
    fl = api.Potential(models["large"], sy.n_atoms, sy.box, 160)(xa, sp)[1]
    fs = api.Potential(models["small"], sy.n_atoms, sy.box, 160)(xa, sp)[1]
    d0 = torch.linalg.vector_norm((fl - fs).double(), dim=0).max().item()
    a.step(xa, va, models["small"], models["large"], 2)
    b.step(xb, vb, None, models["large"], 8)
    n, breach = a.fdiff
    assert n == 2
    assert breach >= d0 * (1 - 1e-6)
    a.step(xa, va, models["small"], models["large"], 2)
    b.step(xb, vb, None, models["large"], 8)
    assert a.fdiff[0] == 4
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    if thermo:
        assert a.o_steps == b.o_steps == 16


def test_no_breach_changes_nothing(models):
    say("monitor: no breach")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a, _ = _state(sy, 4.0, 4)
    b, _ = _state(sy, 4.0, 4)
    a.set_fdiff_threshold(THRESHOLD)
    xa, va = api.to_soa(sy.pos), api.to_soa(v0)
    xb, vb = api.to_soa(sy.pos), api.to_soa(v0)
    a.step(xa, va, models["small"], models["large"], 3)
    b.step(xb, vb, models["small"], models["large"], 3)
    assert a.fdiff == (0, 0.0)
    assert torch.equal(xa, xb) and torch.equal(va, vb)


def test_monitor_rejects_bad_thresholds():
    sy = system("water192")
    st, _ = _state(sy, 2.0, 4)
    for t in (-1.0, float("nan"), float("inf")):
        with pytest.raises(api.DmtsError) as e:
            st.set_fdiff_threshold(t)
        assert e.value.status == api.E_ARG
