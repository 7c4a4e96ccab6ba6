"""Distilling the fast model's readout from the reference model (Methods: training
procedures, system-specific model), checked against the oracle: the design matrix of the
unit-readout models and the reference labels match the oracle's on the same frames, the
fitted readout equals the one the oracle's matrices give for the same ridge problem, and
the distilled model's forces match the oracle's with those weights.  Then what the fit is
for: the distilled RESPA trajectory stays closer to the single-time-step one."""

import numpy as np
import pytest
import torch

from _gpu_common import OP, rel_rmse, say, system, weights, SPECS
from paper_2510_06562_amd import api, distill, synth

pytestmark = pytest.mark.gpu


def _oracle_labels(spec, w, frames, sp, box):
    m = OP.make_model(spec.kind, spec.cutoff, spec.n_rbf, spec.width, w,
                      energy_scale=spec.energy_scale)
    out = [OP.energy_forces(m, x, sp, box) for x in frames]
    return np.concatenate([f.ravel() for _, f, _ in out]), np.array([e[0] for e, _, _ in out])


def _soa_rows(f_flat, n):
    """The library's [3][N] force rows (flattened per frame) as the oracle's (N, 3) rows."""
    return f_flat.reshape(-1, 3, n).transpose(0, 2, 1).ravel()


def test_readout_fit_matches_the_oracle():
    say("distillation vs oracle, water192")
    sy = system("water192")
    n = sy.n_atoms
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    large = api.Model.from_spec(SPECS["large"], weights("large"))
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    snaps = distill.reference_snapshots(large, sp, sy.box, synth.MASSES, sy.pos, v0, 4, 25)
    frames = [api.from_soa(x) for x in snaps]
    ws = weights("small")
    A, Ae = distill.readout_design(synth.SMALL, ws, sp, sy.box, snaps)
    b, be = distill.reference_labels(large, sp, sy.box, snaps)
    # the oracle's design matrix and labels on the same frames
    Ao = np.empty((len(frames) * 3 * n, 64))
    Aeo = np.empty((len(frames), 64))
    for c in range(64):
        w = np.array(ws, dtype=np.float32, copy=True)
        w[-64:] = 0.0
        w[-64 + c] = 1.0
        f, e = _oracle_labels(synth.SMALL, w, frames, sy.species, sy.box)
        Ao[:, c], Aeo[:, c] = f, e
    bo, beo = _oracle_labels(synth.LARGE, weights("large"), frames, sy.species, sy.box)
    A_rows = np.stack([_soa_rows(A[:, c], n) for c in range(64)], axis=1)
    assert rel_rmse(A_rows, Ao) <= 1e-5
    assert rel_rmse(_soa_rows(b, n), bo) <= 1e-5
    assert np.max(np.abs(Ae - Aeo)) <= 1e-5 * np.max(np.abs(Aeo))
    assert np.max(np.abs(be - beo)) <= 1e-7 * n
    # the same ridge problem on the oracle's matrices, written out here
    w0 = np.asarray(ws[-64:], np.float64)
    Aec, bec = Aeo - Aeo.mean(0), beo - beo.mean()
    M = Ao.T @ Ao + (Aec.T @ Aec) / n
    lam = 1e-3 * np.trace(M) / 64
    w_o = np.linalg.solve(M + lam * np.eye(64), Ao.T @ bo + (Aec.T @ bec) / n + lam * w0)
    new, info = distill.fit_readout(synth.SMALL, ws, large, sp, sy.box, snaps)
    say(f"  rms |F_L - F_S| {info['rms_before']:.4f} -> {info['rms_after']:.4f} eV/A, "
        f"|w - w_oracle| / |w_oracle| = {np.linalg.norm(new[-64:] - w_o) / np.linalg.norm(w_o):.1e}")
    assert np.array_equal(new[:-64], ws[:-64])   # only the readout changes
    assert np.linalg.norm(new[-64:] - w_o) <= 1e-4 * np.linalg.norm(w_o)
    assert info["rms_after"] < info["rms_before"]
    # the distilled model, with its float32 weights, on the device and in the oracle
    pot = api.Potential(api.Model.from_spec(synth.SMALL, new), n, sy.box, 128)
    _, F = pot(snaps[-1], sp)
    _, F_o, _ = OP.energy_forces(OP.make_model(0, 3.5, 16, 64, new), frames[-1], sy.species,
                                 sy.box)
    assert rel_rmse(api.from_soa(F), F_o) <= 1e-5


def test_distilled_respa_stays_closer_to_single_time_steps():
    """40 fs of RESPA at 1 fs / 4 fs from the same start with the readout as drawn and as
    fitted, against 40 steps of 1 fs velocity Verlet with the reference model: the fitted
    fast model follows the reference dynamics more closely (RMS position deviation)."""
    say("distilled RESPA vs STS, water192")
    sy = system("water192")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    large = api.Model.from_spec(SPECS["large"], weights("large"))
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    snaps = distill.reference_snapshots(large, sp, sy.box, synth.MASSES, sy.pos, v0, 8, 25)
    ws = weights("small")
    fitted, _ = distill.fit_readout(synth.SMALL, ws, large, sp, sy.box, snaps)

    def run(small, dt, n_inner, n_outer):
        st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128)
        x, v = api.to_soa(sy.pos), api.to_soa(v0)
        st.step(x, v, small, large, n_outer)
        return api.from_soa(x)

    x_sts = run(None, 1.0, 1, 40)
    dev = {}
    for name, w in (("drawn", ws), ("fitted", fitted)):
        x = run(api.Model.from_spec(synth.SMALL, w), 4.0, 4, 10)
        dev[name] = float(np.sqrt(np.mean((x - x_sts) ** 2)))
    say(f"  RMS |x - x_STS| after 40 fs: drawn {dev['drawn']:.2e}, fitted {dev['fitted']:.2e} A")
    assert dev["fitted"] < dev["drawn"]
