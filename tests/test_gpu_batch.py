"""The batched form: 256 uneven open molecules (about 18,000 atoms) evaluated together,
per-molecule energies against the FP64 oracle, launch-shape invariance of the persistent
grid, the autotuner, and equality with a per-molecule loop."""

import numpy as np
import pytest
import torch

from _gpu_common import oracle_ef, rel_rmse, say, system, weights, SPECS
from paper_2510_06562_amd import api

pytestmark = pytest.mark.gpu


def _dev(sy):
    pos = api.to_soa(sy.pos)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    return pos, sp, offs


@pytest.mark.parametrize("prec,ftol", [(api.PREC_FP32, 1e-5), (api.PREC_BF16, 1e-2)])
@pytest.mark.parametrize("which", ["small", "large"])
def test_batch256_matches_oracle_per_molecule(which, prec, ftol):
    say(f"batch256 {which} prec={prec}")
    sy = system("batch256")
    pos, sp, offs = _dev(sy)
    model = api.Model.from_spec(SPECS[which], weights(which), precision=prec)
    pot = api.Potential(model, sy.n_atoms, 0.0, 160, offs)
    E, F = pot(pos, sp)
    E0, F0, _ = oracle_ef("batch256", which)
    sizes = np.diff(sy.sys_offsets)
    assert E.numel() == 256
    err_e = np.abs(E.cpu().numpy() - E0) / sizes
    err_f = rel_rmse(api.from_soa(F), F0)
    say(f"  max |dE|/atom {err_e.max():.2e}, force rel RMSE {err_f:.2e}")
    assert err_f <= ftol
    assert err_e.max() <= (1e-7 if prec == api.PREC_FP32 else 2e-4)


@pytest.mark.parametrize("which", ["small", "large"])
def test_persistent_grid_does_not_change_bits(which):
    say(f"grid invariance {which}")
    sy = system("batch256")
    pos, sp, offs = _dev(sy)
    model = api.Model.from_spec(SPECS[which], weights(which))
    pot = api.Potential(model, sy.n_atoms, 0.0, 160, offs)
    E0, F0 = pot(pos, sp)
    for g in (1, 7, 256, 1024):
        model.grid = g
        E, F = pot(pos, sp)
        assert torch.equal(E, E0) and torch.equal(F, F0), g
    model.grid = 0


def _shapes(which):
    """Every tile shape the model's kernels take (the autotuner's candidates without the
    grid, plus two persistent grids)."""
    if which == "large":
        return [dict(receivers_per_group=nw, atom_tiles=rt, keep_derivatives=1, work_groups=g)
                for nw in (2, 4, 8) for rt in (1, 2) for g in (0, 300)]
    return [dict(receivers_per_group=4, atom_tiles=2, keep_derivatives=k, work_groups=g)
            for k in (0, 1) for g in (0, 300)]


@pytest.mark.parametrize("prec", [api.PREC_FP32, api.PREC_BF16])
@pytest.mark.parametrize("which", ["small", "large"])
def test_every_tile_shape_gives_the_same_bits_and_parity(which, prec):
    """batch256 under every tile shape: bit for bit the default shape's result, which
    matches the oracle per molecule (FP32 1e-5 / BF16 1e-2 force rel. RMSE)."""
    say(f"tile shapes {which} prec={prec}")
    sy = system("batch256")
    pos, sp, offs = _dev(sy)
    model = api.Model.from_spec(SPECS[which], weights(which), precision=prec)
    pot = api.Potential(model, sy.n_atoms, 0.0, 160, offs)
    E0, F0 = pot(pos, sp)
    _, Fo, _ = oracle_ef("batch256", which)
    assert rel_rmse(api.from_soa(F0), Fo) <= (1e-5 if prec == api.PREC_FP32 else 1e-2)
    for sh in _shapes(which):
        model.set_shape(0, **sh)
        assert model.shape(sy.n_atoms) == sh
        E, F = pot(pos, sp)
        assert torch.equal(E, E0) and torch.equal(F, F0), sh


@pytest.mark.parametrize("which", ["small", "large"])
def test_autotune_picks_a_shape_per_size_bucket(which):
    say(f"autotune {which}")
    sy = system("batch256")
    pos, sp, offs = _dev(sy)
    model = api.Model.from_spec(SPECS[which], weights(which), precision=api.PREC_BF16)
    pot = api.Potential(model, sy.n_atoms, 0.0, 160, offs)
    E0, F0 = pot(pos, sp)
    sh, t = api.autotune(pot, pos, sp, reps=2)
    say(f"  chose {sh} at {t:.3f} ms")
    assert t > 0 and sh["work_groups"] in (0, 256, 512, 1024, 2048, 4096)
    assert model.shape(sy.n_atoms) == sh          # cached for this size bucket
    assert model.shape(100) == model.shape(0)     # other buckets keep the default
    E, F = pot(pos, sp)
    assert torch.equal(E, E0) and torch.equal(F, F0)


@pytest.mark.parametrize("which", ["small", "large"])
def test_batched_equals_per_molecule_loop(which):
    """Evaluating each molecule alone gives the same bits as the batched launch."""
    say(f"batched vs loop {which}")
    sy = system("batch256")
    pos, sp, offs = _dev(sy)
    model = api.Model.from_spec(SPECS[which], weights(which))
    pot = api.Potential(model, sy.n_atoms, 0.0, 160, offs)
    E, F = pot(pos, sp)
    F = F.cpu()
    one = api.Potential(model, 200, 0.0, 160)
    for m in range(0, 256, 17):
        a, b = int(sy.sys_offsets[m]), int(sy.sys_offsets[m + 1])
        pm = api.to_soa(sy.pos[a:b])
        sm = sp[a:b].contiguous()
        Em, Fm = one(pm, sm)
        assert Em.item() == E[m].item()
        assert torch.equal(Fm.cpu(), F[:, a:b])


@pytest.mark.parametrize("which", ["small", "large"])
def test_single_system_sum_matches_one_system_batch(which):
    """A large system's energy summed by one work-group per chunk (no system offsets) has
    the same bits as the per-system reduction of a batch holding only that system, and the
    forces do not depend on the offsets either."""
    say(f"energy reduction forms {which}")
    sy = system("batch256")   # all ~18,000 atoms as one open system (several chunks)
    # the molecules are centred at the origin: spread them 30 A apart on a grid, so that the
    # single system has no pairs across molecules (and no row beyond the kernels' caps)
    mol = np.repeat(np.arange(256), np.diff(sy.sys_offsets))
    grid = np.stack([mol % 7, (mol // 7) % 7, mol // 49], axis=1) * 30.0
    pos = api.to_soa(sy.pos + grid)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    model = api.Model.from_spec(SPECS[which], weights(which))
    E1, F1 = api.Potential(model, sy.n_atoms, 0.0, 160)(pos, sp)
    offs = torch.tensor([0, sy.n_atoms], dtype=torch.int32, device="cuda")
    E2, F2 = api.Potential(model, sy.n_atoms, 0.0, 160, offs)(pos, sp)
    assert E1.item() == E2.item()
    assert torch.equal(F1, F2)
