"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element
on the same seeded inputs.

Tolerances (FP32 arithmetic, float64 positions and energy sums):
  * pair sets: exact (integer work);
  * per-atom energies: |E_i - E_i*| <= 1e-5 * max_k |E_k*| and |E - E*| / N <= 1e-7 eV;
  * forces: relative RMSE ||F - F*|| / ||F*|| <= 1e-5 over all 3N components.
"""

import numpy as np
import pytest
import torch

from _gpu_common import oracle_ef, oracle_pairs, rel_rmse, say, system, weights, SPECS
from paper_2510_06562_amd import api

pytestmark = pytest.mark.gpu

E_ATOM_TOL = 1e-5
E_TOTAL_PER_ATOM = 1e-7
F_TOL = 1e-5


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _dev(sy):
    pos = api.to_soa(sy.pos)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    offs = None
    if sy.sys_offsets is not None:
        offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    return pos, sp, offs


def _pairs_of(nl, n):
    offs, nbr, rev = nl.download(n)
    rows = np.repeat(np.arange(n), np.diff(offs))
    real = nbr >= 0
    return offs, nbr, rev, rows, real


@pytest.mark.parametrize("sysname,cut,align", [("water192", 3.5, 4), ("water192", 5.2, 16),
                                               ("water4500", 3.5, 4), ("water4500", 5.2, 16),
                                               ("batch16", 5.2, 16), ("open60", 3.5, 32),
                                               ("wrapped1500", 5.2, 4), ("water21k", 3.5, 4)])
def test_neighbor_set_matches_oracle(sysname, cut, align):
    say(f"nlist {sysname} rc={cut} align={align}")
    sy = system(sysname)
    pos, _, offs_d = _dev(sy)
    nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 200, align)
    nl.build(pos, sy.box, cut, offs_d)
    assert nl.flags() == 0
    offs, nbr, rev, rows, real = _pairs_of(nl, sy.n_atoms)
    assert np.all(offs % align == 0)
    got = set(zip(rows[real].tolist(), nbr[real].tolist()))
    i, j, _ = oracle_pairs(sysname, cut)
    assert got == set(zip(i.tolist(), j.tolist()))
    # padding only at row ends, reverse index points at the mirrored pair
    for a in range(0, sy.n_atoms, max(1, sy.n_atoms // 50)):
        row = nbr[offs[a]:offs[a + 1]]
        k = int(np.sum(row >= 0))
        assert np.all(row[:k] >= 0) and np.all(row[k:] == -1) and len(row) - k < align
    # rows ascend in the sender index
    for a in range(sy.n_atoms):
        row = nbr[offs[a]:offs[a + 1]]
        row = row[row >= 0]
        assert np.all(np.diff(row) > 0)
    p = np.nonzero(real)[0]
    assert np.all(nbr[rev[p]] == rows[p])
    assert np.all(rows[rev[p]] == nbr[p])
    # bitwise reproducible
    nl.build(pos, sy.box, cut, offs_d)
    offs2, nbr2, rev2, _, _ = _pairs_of(nl, sy.n_atoms)
    assert np.array_equal(offs, offs2) and np.array_equal(nbr, nbr2) and np.array_equal(rev, rev2)


@pytest.mark.parametrize("sysname", ["water192", "water21k"])
def test_neighbor_overflow_sets_flag_and_empties_rows(sysname):
    say(f"nlist overflow {sysname}")
    sy = system(sysname)
    pos, _, _ = _dev(sy)
    nl = api.NeighborList(sy.n_atoms, 1000, 4)
    nl.build(pos, sy.box, 5.2)
    assert nl.flags() & api.FLAG_NBR_OVERFLOW
    offs, nbr, rev = nl.download(sy.n_atoms)
    assert np.all(offs == 0)
    assert nl.flags() == 0     # cleared by the previous read


def test_cutoff_above_half_box_is_rejected():
    sy = system("water192")
    pos, _, _ = _dev(sy)
    nl = api.NeighborList(sy.n_atoms, 100000, 4)
    with pytest.raises(api.DmtsError) as e:
        nl.build(pos, sy.box, 6.3)
    assert e.value.status == api.E_BOX


def _check_energy_forces(sysname, which, models):
    sy = system(sysname)
    pos, sp, offs_d = _dev(sy)
    pot = api.Potential(models[which], sy.n_atoms, sy.box, 160, offs_d)
    E, F, Ea = pot(pos, sp, atom_energy=True)
    torch.cuda.synchronize()
    E0, F0, Ea0 = oracle_ef(sysname, which)
    Ea = Ea.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(Ea - Ea0)) <= E_ATOM_TOL * np.max(np.abs(Ea0))
    np.testing.assert_allclose(E.cpu().numpy(), E0, rtol=0, atol=E_TOTAL_PER_ATOM * sy.n_atoms)
    err = rel_rmse(api.from_soa(F), F0)
    say(f"{sysname} {which}: force rel RMSE {err:.2e}, |dE|/N {abs(E.sum().item() - E0.sum()) / sy.n_atoms:.2e}")
    assert err <= F_TOL
    return E, F


@pytest.mark.parametrize("sysname", ["water192", "water4500", "open60", "batch16", "water21k"])
def test_small_model_parity(sysname, models):
    say(f"small model {sysname}")
    _check_energy_forces(sysname, "small", models)


@pytest.mark.parametrize("sysname", ["water192", "water4500", "open60", "batch16"])
def test_large_model_parity(sysname, models):
    say(f"large model {sysname}")
    _check_energy_forces(sysname, "large", models)


@pytest.mark.parametrize("which", ["small", "large"])
def test_forces_are_bitwise_reproducible(which, models):
    say(f"determinism {which}")
    sy = system("water4500")
    pos, sp, _ = _dev(sy)
    pot = api.Potential(models[which], sy.n_atoms, sy.box, 160)
    E1, F1 = pot(pos, sp)
    E2, F2 = pot(pos, sp)
    assert torch.equal(E1, E2) and torch.equal(F1, F2)


def test_pairs_listed_beyond_the_model_cutoff_contribute_nothing(models):
    """A list built with a larger cutoff than the model's gives the same result."""
    say("list cutoff above model cutoff")
    sy = system("water192")
    pos, sp, _ = _dev(sy)
    for which, big in (("small", 5.0), ("large", 6.0)):
        nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 200, 16)
        nl.build(pos, sy.box, big)
        E, F = api.energy_forces(models[which], nl, pos, sp, sy.box)
        E0, F0, _ = oracle_ef("water192", which)
        assert rel_rmse(api.from_soa(F), F0) <= F_TOL
        np.testing.assert_allclose(E.cpu().numpy(), E0, atol=E_TOTAL_PER_ATOM * sy.n_atoms)


def test_reference_model_needs_16_aligned_rows(models):
    sy = system("water192")
    pos, sp, _ = _dev(sy)
    nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 200, 4)
    nl.build(pos, sy.box, 5.2)
    with pytest.raises(api.DmtsError) as e:
        api.energy_forces(models["large"], nl, pos, sp, sy.box)
    assert e.value.status == api.E_ARG


def test_list_below_model_cutoff_is_rejected(models):
    sy = system("water192")
    pos, sp, _ = _dev(sy)
    nl = api.NeighborList(sy.n_atoms, sy.n_atoms * 200, 4)
    nl.build(pos, sy.box, 3.5)
    with pytest.raises(api.DmtsError) as e:
        api.energy_forces(models["large"], nl, pos, sp, sy.box)
    assert e.value.status == api.E_STATE


def test_batched_energies_per_molecule(models):
    say("batch per-molecule energies")
    sy = system("batch16")
    pos, sp, offs_d = _dev(sy)
    for which in ("small", "large"):
        pot = api.Potential(models[which], sy.n_atoms, 0.0, 160, offs_d)
        E, F = pot(pos, sp)
        E0, F0, _ = oracle_ef("batch16", which)
        sizes = np.diff(sy.sys_offsets)
        err = np.abs(E.cpu().numpy() - E0) / sizes
        assert E.numel() == 16 and np.max(err) < E_TOTAL_PER_ATOM


def test_autograd_function_returns_minus_forces(models):
    say("NNPEnergy autograd")
    sy = system("water192")
    pos, sp, _ = _dev(sy)
    pot = api.Potential(models["small"], sy.n_atoms, sy.box, 160)
    x = pos.clone().requires_grad_(True)
    E = api.NNPEnergy.apply(x, pot, sp)
    E.sum().backward()
    _, F0, _ = oracle_ef("water192", "small")
    assert rel_rmse(-api.from_soa(x.grad), F0) <= F_TOL


def _gpu_fd(pot, pos, sp, comps, h):
    out = []
    for a, c in comps:
        xp = pos.clone()
        xp[c, a] += h
        xm = pos.clone()
        xm[c, a] -= h
        ep = pot(xp, sp, want_forces=False)[0].item()
        em = pot(xm, sp, want_forces=False)[0].item()
        out.append(-(ep - em) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("which", ["small", "large"])
def test_gpu_forces_match_gpu_finite_differences(which, models):
    """Central differences of the device energy itself on sampled components.

    The device energy is a sum of float32 per-atom energies whose readout adds 64 terms
    of magnitude ~0.5 (before the 0.01 eV scale): each E_i carries ~3e-9 eV of rounding,
    ~20 of them change when one atom moves, so a difference quotient over 2h = 2e-4 A
    has ~1e-4 eV/A of noise (~5% of a typical force).  At h = 3e-3 A the noise is ~0.3%
    and the O(h^2) truncation ~1e-4 (radial basis width 0.23 A), so that step carries the
    1e-2 bound; h = 1e-4 A keeps a loose bound.  The tight check of the analytic forces is
    the comparison with the oracle's gradient (1e-5)."""
    say(f"GPU finite differences {which}")
    sy = system("water192")
    pos, sp, _ = _dev(sy)
    pot = api.Potential(models[which], sy.n_atoms, sy.box, 160)
    _, F = pot(pos, sp)
    F = api.from_soa(F)
    rng = np.random.default_rng(11)
    comps = [(int(rng.integers(sy.n_atoms)), int(rng.integers(3))) for _ in range(24)]
    an = np.array([F[a, c] for a, c in comps])
    fd = _gpu_fd(pot, pos, sp, comps, 3e-3)
    assert np.linalg.norm(fd - an) / np.linalg.norm(an) < 1e-2
    fd4 = _gpu_fd(pot, pos, sp, comps, 1e-4)
    assert np.linalg.norm(fd4 - an) / np.linalg.norm(an) < 0.25
