"""The force-difference monitor: when |F - F_small| of an atom exceeds the threshold, a
dmts_step call is redone as single-time-step steps of the inner length with the reference
model (the paper's temporary reversion to STS integration).  The threshold is forced from
the host: a tiny one makes every call breach, a huge one none."""

import numpy as np
import pytest
import torch

from _gpu_common import say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _state(sy, dt, n_inner):
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    return api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128), sp


@pytest.mark.parametrize("thermo", [False, True])
def test_breach_redoes_the_call_as_single_time_steps(models, thermo):
    """With a threshold below every force difference each call is redone, and the
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
    n, breach = a.fdiff   # the largest breach seen by the (rolled back) first attempt
    assert n == 1
    assert breach >= d0 * (1 - 1e-6)
    a.step(xa, va, models["small"], models["large"], 2)
    b.step(xb, vb, None, models["large"], 8)
    assert a.fdiff[0] == 2
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    if thermo:
        assert a.o_steps == b.o_steps == 16


def test_no_breach_changes_nothing(models):
    say("monitor: no breach")
    sy = system("water192")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    a, _ = _state(sy, 4.0, 4)
    b, _ = _state(sy, 4.0, 4)
    a.set_fdiff_threshold(6.505)   # 150 kcal/mol/A
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
