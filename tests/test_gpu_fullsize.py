"""Parity at the full size of the 100,001-atom solvated workload: both models, FP32 and BF16,
evaluated on the whole system on one list built at the reference cutoff (5.2 A, rows
aligned to 16), as the DMTS step shares it; the per-atom energies and forces of sixteen
sampled atoms (chain and water) are compared with oracle values stored by
tests/golden/make_solvated100k_samples.py, which evaluates the oracle on the open cluster
holding each atom's receptive field.

Tolerances as in the smaller parity tests: FP32 per-atom energies within 1e-5 of the
largest sampled |E_i*| and forces within 1e-5 relative RMSE over the sampled components;
BF16 energies within 2e-4 eV per atom and forces within 1e-2."""

import json
import os

import numpy as np
import pytest
import torch

from _gpu_common import say, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def c4():
    say("solvated100k: system")
    sy = synth.solvated_chain()
    with open(os.path.join(HERE, "golden", "solvated100k_samples.json")) as f:
        ref = json.load(f)
    assert ref["n_atoms"] == sy.n_atoms
    pos = api.to_soa(sy.pos)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 96, 16)
    nl.build(pos, sy.box, 5.2)
    assert nl.flags() == 0
    return sy, ref, pos, sp, nl


@pytest.mark.parametrize("prec", [api.PREC_FP32, api.PREC_BF16])
@pytest.mark.parametrize("which", ["small", "large"])
def test_solvated100k_sampled_parity(c4, which, prec):
    sy, ref, pos, sp, nl = c4
    say(f"solvated100k {which} prec={prec}")
    model = api.Model.from_spec(SPECS[which], weights(which), precision=prec)
    _, F, Ea = api.energy_forces(model, nl, pos, sp, sy.box, atom_energy=True)
    torch.cuda.synchronize()
    atoms = ref["atoms"]
    e_ref = np.asarray(ref["energy"][which])
    e_gpu = Ea.cpu().numpy().astype(np.float64)[atoms]
    fa = ref["force_atoms"][which]
    f_ref = np.asarray(ref["force"][which])
    f_gpu = F.cpu().numpy().astype(np.float64)[:, fa].T
    de = np.max(np.abs(e_gpu - e_ref))
    ferr = np.linalg.norm(f_gpu - f_ref) / np.linalg.norm(f_ref)
    say(f"  max |dE_i| {de:.2e} eV, sampled force rel RMSE {ferr:.2e}")
    assert np.all(np.isfinite(F.cpu().numpy()))
    if prec == api.PREC_FP32:
        assert de <= 1e-5 * np.max(np.abs(e_ref))
        assert ferr <= 1e-5
    else:
        assert de <= 2e-4
        assert ferr <= 1e-2
