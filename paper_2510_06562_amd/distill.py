"""Distillation of the fast model from the reference model (the paper trains its fast model
on energies and forces of frames from a short molecular-dynamics run of the reference model;
Methods: training procedures, system-specific model), here on synthetic frames, with the
weights the library evaluates.

Only the fast model's readout vector w2 (the last `width` entries of its weight blob) is
fitted.  The model's energy E = s_E sum_i w2 . SiLU(W1 h_i) is linear in w2, and so are its
forces: with E^(c), F^(c) the energy and forces of the same model with w2 = e_c,
E(w2) = sum_c w2_c E^(c) and F(w2) = sum_c w2_c F^(c).  The `width` models with unit
readouts give a design matrix over the frames; a ridge least-squares fit toward the original
readout matches the reference forces and, with a weight, the reference energies relative to
their mean over the frames (an energy offset between the two models is invisible to the
dynamics).  Every energy and force evaluation runs in the library's kernels; the fit is a
`width`-unknown linear solve on the host.  The training loop stays here, outside the
library.
"""

from __future__ import annotations

import numpy as np
import torch

from . import api


def reference_snapshots(large: api.Model, species: torch.Tensor, box: float, masses,
                        pos0: np.ndarray, v0: np.ndarray, n_snap: int, stride: int,
                        dt_fs: float = 1.0, atom_masses=None) -> list:
    """Positions ([3][N] float64 device tensors) every `stride` steps of a single-time-step
    run of `dt_fs` with the reference model from (pos0, v0); `atom_masses` (per atom, amu)
    replaces the species masses when the run uses repartitioned ones."""
    n = pos0.shape[0]
    st = api.DMTS(n, box, species, masses, dt_fs, 1, 64, 128)
    if atom_masses is not None:
        st.set_atom_masses(atom_masses)
    x, v = api.to_soa(pos0), api.to_soa(v0)
    out = []
    for _ in range(n_snap):
        st.step(x, v, None, large, stride)
        out.append(x.clone())
    return out


def readout_design(spec, weights: np.ndarray, species: torch.Tensor, box: float,
                   snapshots: list, precision: int = api.PREC_FP32):
    """(A, Ae): column c of A is the forces (stacked over the frames, float64) and row s of
    Ae the energies (frame s) of the fast model with its readout vector replaced by e_c."""
    F = spec.width
    n = snapshots[0].shape[1]
    # one list per frame, shared by the unit-readout models
    lists = []
    for x in snapshots:
        nl = api.NeighborList(n, n * (128 + 16), 16)
        nl.build(x, box, spec.cutoff)
        lists.append(nl)
    A = np.empty((len(snapshots) * 3 * n, F), dtype=np.float64)
    Ae = np.empty((len(snapshots), F), dtype=np.float64)
    for c in range(F):
        w = np.array(weights, dtype=np.float32, copy=True)
        w[-F:] = 0.0
        w[-F + c] = 1.0
        model = api.Model.from_spec(spec, w, precision=precision)
        for s, (x, nl) in enumerate(zip(snapshots, lists)):
            e, f = api.energy_forces(model, nl, x, species, box)
            A[s * 3 * n:(s + 1) * 3 * n, c] = f.double().cpu().numpy().ravel()
            Ae[s, c] = e.item()
    return A, Ae


def reference_labels(large: api.Model, species: torch.Tensor, box: float, snapshots: list):
    """(forces stacked over the frames, energies per frame) of the reference model."""
    n = snapshots[0].shape[1]
    pot = api.Potential(large, n, box, 128)
    f, e = [], []
    for x in snapshots:
        E, F = pot(x, species)
        f.append(F.double().cpu().numpy().ravel())
        e.append(E.item())
    return np.concatenate(f), np.array(e)


def reference_forces(large: api.Model, species: torch.Tensor, box: float,
                     snapshots: list) -> np.ndarray:
    return reference_labels(large, species, box, snapshots)[0]


def solve_readout(A, Ae, b, be, w0, n_atoms: int, ridge: float = 1e-3,
                  energy_weight: float = 1.0) -> np.ndarray:
    """argmin_w |A w - b|^2 + (energy_weight^2 / n_atoms) |Ae' w - be'|^2 + lam |w - w0|^2,
    Ae', be' the energies minus their mean over the frames, lam = ridge times the mean
    diagonal of the normal matrix."""
    Aec = Ae - Ae.mean(axis=0)
    bec = be - be.mean()
    we2 = energy_weight ** 2 / n_atoms
    M = A.T @ A + we2 * (Aec.T @ Aec)
    lam = ridge * float(np.trace(M)) / M.shape[0]
    return np.linalg.solve(M + lam * np.eye(M.shape[0]), A.T @ b + we2 * (Aec.T @ bec) + lam * w0)


def fit_readout(spec, weights: np.ndarray, large: api.Model, species: torch.Tensor,
                box: float, snapshots: list, ridge: float = 1e-3,
                precision: int = api.PREC_FP32, energy_weight: float = 1.0):
    """The fast model's weights with the readout vector fitted to the reference energies and
    forces on `snapshots`.  Returns (weights, info) with the RMS force difference before and
    after on the fitting set."""
    F = spec.width
    A, Ae = readout_design(spec, weights, species, box, snapshots, precision)
    b, be = reference_labels(large, species, box, snapshots)
    n = snapshots[0].shape[1]
    w0 = np.asarray(weights[-F:], dtype=np.float64)
    w = solve_readout(A, Ae, b, be, w0, n, ridge, energy_weight)
    out = np.array(weights, dtype=np.float32, copy=True)
    out[-F:] = w.astype(np.float32)
    rms = lambda r: float(np.sqrt(np.mean(r * r)))  # noqa: E731
    ec = lambda e: e - e.mean()  # noqa: E731
    info = {"rms_before": rms(A @ w0 - b), "rms_after": rms(A @ w - b),
            "rms_reference": rms(b), "n_forces": int(b.size), "frames": len(snapshots),
            "energy_rms_per_atom_before": rms(ec(Ae @ w0) - ec(be)) / n,
            "energy_rms_per_atom_after": rms(ec(Ae @ w) - ec(be)) / n}
    return out, info


def slow_force_autocorrelation(large: api.Model, small: api.Model, species: torch.Tensor,
                               box: float, masses, pos0: np.ndarray, v0: np.ndarray,
                               n_frames: int, dt_fs: float = 1.0, atom_masses=None) -> dict:
    """How slow the slow force is: along a single-time-step run of the reference model,
    the normalized autocorrelation C(tau) = <dF(t) . dF(t + tau)> / <dF . dF> of
    dF = F_large - F_small, its integrated time dt (1/2 + sum_{tau >= 1} C(tau)) up to the
    first negative C, the lag of the first zero, and the RMS of dF per component."""
    n = pos0.shape[0]
    st = api.DMTS(n, box, species, masses, dt_fs, 1, 64, 128)
    if atom_masses is not None:
        st.set_atom_masses(atom_masses)
    pl = api.Potential(large, n, box, 128)
    ps = api.Potential(small, n, box, 128)
    x, v = api.to_soa(pos0), api.to_soa(v0)
    d = []
    for _ in range(n_frames):
        d.append((pl(x, species)[1] - ps(x, species)[1]).double().cpu().numpy().ravel())
        st.step(x, v, None, large, 1)
    D = np.array(d)
    c0 = float(np.mean(np.sum(D * D, axis=1)))
    C = [1.0]
    for lag in range(1, n_frames // 2):
        C.append(float(np.mean(np.sum(D[:-lag] * D[lag:], axis=1))) / c0)
    C = np.array(C)
    neg = np.nonzero(C < 0.0)[0]
    cut = int(neg[0]) if len(neg) else len(C)
    tau = dt_fs * (0.5 + float(np.sum(C[1:cut])))
    return {"tau_int_fs": tau, "first_zero_fs": cut * dt_fs if len(neg) else None,
            "C_at_1fs": float(C[1]) if len(C) > 1 else None,
            "C_at_4fs": float(C[int(round(4 / dt_fs))]) if len(C) > int(round(4 / dt_fs)) else None,
            "rms_dF": float(np.sqrt(c0 / D.shape[1])), "frames": n_frames}
