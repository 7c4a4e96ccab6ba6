"""Edge cases of the HIP path against the FP64 oracle: capacity overflows that must be
reported (never silently truncated), an isolated atom, pairs just inside the cutoff,
element-wise per-atom energies of the BF16 form, and the batched form under autograd."""

import numpy as np
import pytest
import torch

from _gpu_common import OP, oracle_ef, oracle_model, rel_rmse, say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _ball(n, radius, seed):
    """n atoms uniformly in a ball (open boundaries), random species."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v *= (radius * rng.uniform(0, 1, n) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
    return v, rng.integers(0, 5, n).astype(np.int32)


def _dev(pos, sp):
    return api.to_soa(pos), torch.as_tensor(sp, dtype=torch.int32, device="cuda")


def test_fast_pair_cap_overflow_is_reported(models):
    """100 atoms within 2.5 A: every atom has more than 64 pairs inside 3.5 A, more than the
    fast kernels hold per atom.  Energy+forces raise E_CAPACITY (the list's flag word), and
    a RESPA call on the same atoms returns DMTS_E_CAPACITY."""
    say("cap: fast model 64 pairs per atom")
    pos, sp = _ball(100, 2.5, 1)
    i, _, _ = OP._pairs(pos, 0.0, 3.5, None)
    assert np.bincount(i, minlength=100).max() > 64
    x, s = _dev(pos, sp)
    pot = api.Potential(models["small"], 100, 0.0, 120)
    with pytest.raises(api.DmtsError) as e:
        pot(x, s)
    assert e.value.status == api.E_CAPACITY
    pot.check = False
    pot(x, s)
    assert pot.nlist.flags() & api.FLAG_NBR_OVERFLOW
    st = api.DMTS(100, 0.0, s, synth.MASSES, 2.0, 2, 120, 120)
    v = torch.zeros_like(x)
    with pytest.raises(api.DmtsError) as e:
        st.step(x, v, models["small"], models["large"], 1)
    assert e.value.status == api.E_CAPACITY


def test_list_row_cap_overflow_is_reported(models):
    """300 atoms within 2.6 A: every row of the 5.2 A list holds 299 senders, more than the
    256 a row can take.  The list build and the reference model raise E_CAPACITY."""
    say("cap: neighbor row 256 entries")
    pos, sp = _ball(300, 2.6, 2)
    x, s = _dev(pos, sp)
    pot = api.Potential(models["large"], 300, 0.0, 320)
    with pytest.raises(api.DmtsError) as e:
        pot(x, s)
    assert e.value.status == api.E_CAPACITY
    nl = api.NeighborList(300, 300 * 336, 16)
    nl.build(x, 0.0, 5.2)
    assert nl.flags() & api.FLAG_NBR_OVERFLOW


@pytest.mark.parametrize("which", ["small", "large"])
def test_isolated_atom_and_pairs_at_the_cutoff(which, models):
    """An open system: a water trimer, an atom 30 A away from everything (E_i = 0 and F_i = 0
    exactly: no biases, SiLU(0) = 0), and a dimer at r_c (1 - 1e-6), whose pair is inside
    the cutoff by 1e-6 r_c and contributes f_c ~ 1e-11 of a message.  Per-atom energies and
    forces against the oracle."""
    say(f"isolated atom and r_c(1 - 1e-6) pair {which}")
    rc = SPECS[which].cutoff
    water = np.array([[0.0, 0.0, 0.0], [0.96, 0.0, 0.0], [-0.24, 0.93, 0.0]])
    trimer = np.vstack([water, water @ synth.random_rotation(1).T + [2.8, 0.4, 0.3],
                        water @ synth.random_rotation(2).T + [0.5, 2.9, -0.6]])
    pos = np.vstack([trimer, [[30.0, 0.0, 0.0]],
                     [[0.0, 30.0, 0.0], [0.0, 30.0 + rc * (1 - 1e-6), 0.0]]])
    sp = np.array([3, 0, 0] * 3 + [4, 1, 2], dtype=np.int32)
    x, s = _dev(pos, sp)
    pot = api.Potential(models[which], len(pos), 0.0, 64)
    E, F, Ea = pot(x, s, atom_energy=True)
    E0, F0, Ea0 = OP.energy_forces(oracle_model(which), pos, sp, 0.0)
    Ea, F = Ea.cpu().numpy().astype(np.float64), api.from_soa(F)
    assert Ea[9] == 0.0 and np.all(F[9] == 0.0)
    assert np.max(np.abs(Ea - Ea0)) <= 1e-5 * np.max(np.abs(Ea0))
    assert rel_rmse(F[:9], F0[:9]) <= 1e-5
    # the dimer's energy is ~1e-11 of a message: both sides agree to far below FP32 noise
    assert np.max(np.abs(Ea[10:] - Ea0[10:])) <= 1e-9
    assert np.max(np.abs(F[10:] - F0[10:])) <= 1e-7


@pytest.mark.parametrize("which", ["small", "large"])
def test_bf16_per_atom_energies_within_rounding_bound(which):
    """Element-wise per-atom energies of the BF16 form.  Every operand entering a BF16
    product is rounded to 8 significant bits (relative error <= 2^-9); through the pair
    contraction, the message sums and the readout chain the error of E_i stays a small
    multiple of 2^-9 times the size of the readout terms, s_E sum_c |w_c SiLU(z_c)| (from
    the oracle), which does not shrink when the terms cancel.  Bound: 8 units of 2^-9 of
    that size (four chained roundings: radial operands, message sums into the readout,
    readout operands, and for the reference model the update chains; twice that for
    margin).  Measured on the 4,500-atom box: at most 1.0 (fast) and 1.8 (reference)."""
    say(f"bf16 per-atom energies {which}")
    sy = system("water4500")
    model = api.Model.from_spec(SPECS[which], weights(which), precision=api.PREC_BF16)
    x, s = _dev(sy.pos, sy.species)
    _, _, Ea = api.Potential(model, sy.n_atoms, sy.box, 160)(x, s, atom_energy=True)
    _, _, Ea0 = oracle_ef("water4500", which)
    size = OP.readout_magnitude(oracle_model(which), sy.pos, sy.species, sy.box)
    ratio = np.abs(Ea.cpu().numpy().astype(np.float64) - Ea0) / (2.0 ** -9 * size)
    say(f"  max |dE_i| / (2^-9 size_i) = {ratio.max():.2f}, median {np.median(ratio):.3f}")
    assert ratio.max() <= 8.0


@pytest.mark.parametrize("which", ["small", "large"])
def test_autograd_batched_weights_per_molecule(which, models):
    """NNPEnergy on a batch of 16 molecules with a different weight per molecule: the
    gradient of sum_s w_s E_s is -w_s F_i for the atoms of molecule s."""
    say(f"NNPEnergy batched {which}")
    sy = system("batch16")
    x, s = _dev(sy.pos, sy.species)
    offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    pot = api.Potential(models[which], sy.n_atoms, 0.0, 160, offs)
    wts = torch.linspace(-2.0, 3.0, 16, dtype=torch.float64, device="cuda")
    xr = x.clone().requires_grad_(True)
    E = api.NNPEnergy.apply(xr, pot, s)
    (E * wts).sum().backward()
    _, F0, _ = oracle_ef("batch16", which)
    g_atom = np.repeat(wts.cpu().numpy(), np.diff(sy.sys_offsets))
    assert rel_rmse(-api.from_soa(xr.grad), F0 * g_atom[:, None]) <= 1e-5
