"""The allocation-free entry point nnp_energy_forces_noalloc (fixed device scratch array)
against nnp_energy_forces on the same inputs: two calls in a row, the second on a smaller
system, each bit for bit equal to the allocating entry point; and its limits."""

import numpy as np
import pytest
import torch

from _gpu_common import say, system, weights, SPECS
from paper_2510_06562_amd import api

pytestmark = pytest.mark.gpu


def _inputs(sy, n):
    pos = api.to_soa(sy.pos[:n])
    sp = torch.as_tensor(sy.species[:n], dtype=torch.int32, device="cuda")
    return pos, sp


@pytest.mark.parametrize("prec", [api.PREC_FP32, api.PREC_BF16])
def test_noalloc_equals_allocating_entry_point_twice(prec):
    say(f"noalloc vs nnp_energy_forces, prec {prec}")
    model = api.Model.from_spec(SPECS["small"], weights("small"), precision=prec)
    big = system("water4500")
    small_open = system("open60")
    cases = [(big, big.n_atoms, big.box), (small_open, small_open.n_atoms, 0.0)]
    nl = api.NeighborList(big.n_atoms, big.n_atoms * 200, 16)
    for sy, n, box in cases:   # the second call is on a smaller input
        pos, sp = _inputs(sy, n)
        nl.build(pos, box, 3.5)
        E0, F0, Ea0 = api.energy_forces(model, nl, pos, sp, box, atom_energy=True)
        E = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        F = torch.full((3, n), float("nan"), dtype=torch.float32, device="cuda")
        Ea = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        api.energy_forces_noalloc(model, nl, pos, sp, box, E, F, Ea)
        torch.cuda.synchronize()
        assert nl.flags() == 0
        assert torch.equal(E, E0) and torch.equal(F, F0) and torch.equal(Ea, Ea0), n


def test_noalloc_rejects_what_it_cannot_hold():
    say("noalloc limits")
    sy = system("water21k")
    n = 9000                                   # above the 8,192-atom scratch limit
    model = api.Model.from_spec(SPECS["small"], weights("small"))
    pos, sp = _inputs(sy, n)
    nl = api.NeighborList(n, n * 200, 16)
    nl.build(pos, 0.0, 3.5)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(api.DmtsError) as e:
        api.energy_forces_noalloc(model, nl, pos, sp, 0.0, E)
    assert e.value.status == api.E_CAPACITY
    large = api.Model.from_spec(SPECS["large"], weights("large"))
    pos, sp = _inputs(sy, 100)
    nl.build(pos, 0.0, 5.2)
    with pytest.raises(api.DmtsError) as e:
        api.energy_forces_noalloc(large, nl, pos, sp, 0.0, E)
    assert e.value.status == api.E_ARG


def test_noalloc_batched_molecules():
    say("noalloc batch16")
    sy = system("batch16")
    model = api.Model.from_spec(SPECS["small"], weights("small"))
    pos, sp = _inputs(sy, sy.n_atoms)
    offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 200, 16)
    nl.build(pos, 0.0, 3.5, offs)
    E0, F0 = api.energy_forces(model, nl, pos, sp, 0.0, offs)
    E = torch.zeros(16, dtype=torch.float64, device="cuda")
    F = torch.zeros((3, sy.n_atoms), dtype=torch.float32, device="cuda")
    api.energy_forces_noalloc(model, nl, pos, sp, 0.0, E, F, sys_offsets=offs)
    assert torch.equal(E, E0) and torch.equal(F, F0)
    assert np.isfinite(E.cpu().numpy()).all()
