"""The BF16 form: MLP contractions with bfloat16 operands (nearest even) and FP32
accumulation, FP32 geometry, float64 positions and energy sums.  Forces must stay within
1e-2 relative RMSE of the FP64 oracle; per-atom energy errors are reported and bounded."""

import numpy as np
import pytest
import torch

from _gpu_common import oracle_ef, rel_rmse, say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu

F_TOL_BF16 = 1e-2
E_TOL_BF16 = 2e-4   # eV per atom


@pytest.fixture(scope="module")
def models16():
    return {k: api.Model.from_spec(SPECS[k], weights(k), precision=api.PREC_BF16)
            for k in ("small", "large")}


def _dev(sy):
    pos = api.to_soa(sy.pos)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    offs = None
    if sy.sys_offsets is not None:
        offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    return pos, sp, offs


@pytest.mark.parametrize("which", ["small", "large"])
@pytest.mark.parametrize("sysname", ["water192", "water4500", "open60", "batch16"])
def test_bf16_parity(sysname, which, models16):
    say(f"bf16 {which} {sysname}")
    sy = system(sysname)
    pos, sp, offs = _dev(sy)
    pot = api.Potential(models16[which], sy.n_atoms, sy.box, 160, offs)
    E, F = pot(pos, sp)
    E0, F0, _ = oracle_ef(sysname, which)
    err = rel_rmse(api.from_soa(F), F0)
    dE = np.max(np.abs(E.cpu().numpy() - E0)) / sy.n_atoms
    say(f"  force rel RMSE {err:.2e}, |dE|/N {dE:.2e} eV")
    assert err <= F_TOL_BF16
    assert dE <= E_TOL_BF16


@pytest.mark.parametrize("which", ["small", "large"])
def test_bf16_is_bitwise_reproducible(which, models16):
    sy = system("water4500")
    pos, sp, _ = _dev(sy)
    pot = api.Potential(models16[which], sy.n_atoms, sy.box, 160)
    E1, F1 = pot(pos, sp)
    E2, F2 = pot(pos, sp)
    assert torch.equal(E1, E2) and torch.equal(F1, F2)


def test_bf16_dmts_short_nve(models16):
    """DMTS 1 fs / 4 fs with both BF16 models on the 4,500-atom box: the conserved energy
    stays within 1e-4 eV per atom over 400 fs."""
    say("bf16 DMTS NVE water4500")
    sy = system("water4500")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, 4.0, 4)
    x = api.to_soa(sy.pos)
    v = api.to_soa(synth.maxwell_boltzmann(sy.species, 300.0, 201))
    H = [st.step(x, v, models16["small"], models16["large"], 10)[3].item() for _ in range(10)]
    assert np.max(np.abs(np.array(H) - H[0])) / sy.n_atoms < 1e-4
