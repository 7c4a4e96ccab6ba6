"""Distillation of the fast model from the reference model (the paper trains its fast model
on the reference model's forces; here on synthetic snapshots, with the weights the
library evaluates).

Only the fast model's readout vector w2 (the last `width` entries of its weight blob) is
fitted.  The model's energy E = s_E sum_i w2 . SiLU(W1 h_i) is linear in w2, and so are its
forces: with F^(c) the forces of the same model with w2 = e_c, F(w2) = sum_c w2_c F^(c).
The `width` models with unit readouts give a design matrix over the snapshots, and a ridge
least-squares fit toward the original readout matches the reference forces.  Every force
evaluation runs in the library's kernels; the fit is a `width`-unknown linear solve on the
host.  The training loop stays here, outside the library.
"""

from __future__ import annotations

import numpy as np
import torch

from . import api


def reference_snapshots(large: api.Model, species: torch.Tensor, box: float, masses,
                        pos0: np.ndarray, v0: np.ndarray, n_snap: int, stride: int,
                        dt_fs: float = 1.0) -> list:
    """Positions ([3][N] float64 device tensors) every `stride` steps of a single-time-step
    run of `dt_fs` with the reference model from (pos0, v0)."""
    n = pos0.shape[0]
    st = api.DMTS(n, box, species, masses, dt_fs, 1, 64, 128)
    x, v = api.to_soa(pos0), api.to_soa(v0)
    out = []
    for _ in range(n_snap):
        st.step(x, v, None, large, stride)
        out.append(x.clone())
    return out


def readout_design(spec, weights: np.ndarray, species: torch.Tensor, box: float,
                   snapshots: list, precision: int = api.PREC_FP32) -> np.ndarray:
    """Columns c = forces (stacked over snapshots, float64) of the fast model with its
    readout vector replaced by the unit vector e_c."""
    F = spec.width
    n = snapshots[0].shape[1]
    # one list per snapshot, shared by the unit-readout models
    lists = []
    for x in snapshots:
        nl = api.NeighborList(n, n * (128 + 16), 16)
        nl.build(x, box, spec.cutoff)
        lists.append(nl)
    cols = np.empty((len(snapshots) * 3 * n, F), dtype=np.float64)
    for c in range(F):
        w = np.array(weights, dtype=np.float32, copy=True)
        w[-F:] = 0.0
        w[-F + c] = 1.0
        model = api.Model.from_spec(spec, w, precision=precision)
        for s, (x, nl) in enumerate(zip(snapshots, lists)):
            f = api.energy_forces(model, nl, x, species, box)[1]
            cols[s * 3 * n:(s + 1) * 3 * n, c] = f.double().cpu().numpy().ravel()
    return cols


def reference_forces(large: api.Model, species: torch.Tensor, box: float,
                     snapshots: list) -> np.ndarray:
    n = snapshots[0].shape[1]
    pot = api.Potential(large, n, box, 128)
    return np.concatenate([pot(x, species)[1].double().cpu().numpy().ravel() for x in snapshots])


def fit_readout(spec, weights: np.ndarray, large: api.Model, species: torch.Tensor,
                box: float, snapshots: list, ridge: float = 1e-3,
                precision: int = api.PREC_FP32):
    """The fast model's weights with the readout vector fitted to the reference forces on
    `snapshots` (ridge toward the original readout, weighted by `ridge` times the mean
    diagonal of A^T A).  Returns (weights, info) with the RMS force difference before and
    after on the fitting set."""
    F = spec.width
    A = readout_design(spec, weights, species, box, snapshots, precision)
    b = reference_forces(large, species, box, snapshots)
    w0 = np.asarray(weights[-F:], dtype=np.float64)
    AtA = A.T @ A
    lam = ridge * float(np.trace(AtA)) / F
    w = np.linalg.solve(AtA + lam * np.eye(F), A.T @ b + lam * w0)
    out = np.array(weights, dtype=np.float32, copy=True)
    out[-F:] = w.astype(np.float32)
    rms = lambda r: float(np.sqrt(np.mean(r * r)))  # noqa: E731
    info = {"rms_before": rms(A @ w0 - b), "rms_after": rms(A @ w - b),
            "rms_reference": rms(b), "n_forces": int(b.size)}
    return out, info
