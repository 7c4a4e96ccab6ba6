"""Distilling the fast model's readout from the reference model: the fast model's forces
are linear in its readout vector (checked against the design matrix), and the fitted
readout brings the fast forces closer to the reference forces on the fitting snapshots
and on a held-out snapshot of the same reference-model run."""

import numpy as np
import pytest
import torch

from _gpu_common import say, system, weights, SPECS
from paper_2510_06562_amd import api, distill, synth

pytestmark = pytest.mark.gpu


def _rms(a):
    return float(np.sqrt(np.mean(np.asarray(a, np.float64) ** 2)))


def test_readout_distillation_water192():
    say("distill the fast readout, water192")
    sy = system("water192")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    large = api.Model.from_spec(SPECS["large"], weights("large"))
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    snaps = distill.reference_snapshots(large, sp, sy.box, synth.MASSES, sy.pos, v0, 4, 25)
    fit, held = snaps[:3], snaps[3:]
    ws = weights("small")
    new, info = distill.fit_readout(synth.SMALL, ws, large, sp, sy.box, fit)
    say(f"  fit set: rms |F_L - F_S| {info['rms_before']:.4f} -> {info['rms_after']:.4f} eV/A "
        f"(|F_L| {info['rms_reference']:.4f})")
    assert info["rms_after"] < info["rms_before"]
    assert np.array_equal(new[:-64], ws[:-64])   # only the readout changes

    f_l = distill.reference_forces(large, sp, sy.box, held)

    def fast_forces(w):
        pot = api.Potential(api.Model.from_spec(synth.SMALL, w), sy.n_atoms, sy.box, 128)
        return pot(held[0], sp)[1].double().cpu().numpy().ravel()
    before, after = _rms(fast_forces(ws) - f_l), _rms(fast_forces(new) - f_l)
    say(f"  held out: {before:.4f} -> {after:.4f} eV/A")
    assert after < before
    # linearity in the readout: the distilled model's forces are the design matrix times
    # its readout vector
    A = distill.readout_design(synth.SMALL, ws, sp, sy.box, held)
    f_new = fast_forces(new)
    pred = A @ new[-64:].astype(np.float64)
    assert np.linalg.norm(pred - f_new) <= 1e-5 * np.linalg.norm(f_new)
