"""The two synthetic neural network potentials, energy and analytic forces in FP64
(oracle; test infrastructure only).

The paper pairs a cheap distilled model (one message-passing interaction, 3.5 A
receptive field) with an expensive reference model (two message-passing interactions,
~11 A receptive field) (Methods: neural network architectures; Abstract).  Its trained
architectures and weights are not available, so both levels are defined here as explicit
synthetic models with the same structure:

Shared pieces (for a pair i <- j, d = d_ij, r = |d|, cutoff r_c, K radial functions):
    b_k(r)  = exp(-(r - mu_k)^2 / (2 sigma^2)),   mu_k = k r_c/(K-1),  sigma = r_c/(K-1)
    f_c(r)  = (cos(pi r / r_c) + 1) / 2  for r < r_c, else 0
    SiLU(t) = t / (1 + exp(-t))
    e_z     = row z of a species embedding table (5 species x 16)

One-interaction model (kind 0; fast level):
    a_ij = W_pair [ b(r_ij) ; e_{z_i} ; e_{z_j} ]         (receiver block, then sender)
    m_ij = f_c(r_ij) * SiLU(a_ij)
    h_i  = sum_{j in N(i)} m_ij
    E_i  = s_E * w_atom2 . SiLU(W_atom1 h_i)
    E    = sum_i E_i

Two-interaction model (kind 1; reference level), with u_ij = d_ij / r_c and the
traceless second moment Y2(u) = u u^T - |u|^2 I / 3:
    layer t:  a^t_ij = W_pair_t [ b(r_ij) ; s^t_i ; s^t_j ],  s^1 = e_z,  s^2 = h^1
              m^t_ij = f_c(r_ij) * SiLU(a^t_ij)
              M0_i = sum_j m_ij,  M1_i = sum_j m_ij (x) u_ij,  M2_i = sum_j m_ij (x) Y2(u_ij)
              q_i  = [ M0_i ; sum_a M1_{i,c,a}^2 ; sum_ab M2_{i,c,ab}^2 ]   (channel-wise)
    h^1_i = SiLU(U1 q^1_i);   h^2_i = h^1_i + SiLU(U2 q^2_i)
    E_i   = s_E * w_out2 . SiLU(W_out1 h^2_i)

No biases.  Forces are F_i = -dE/dx_i, computed by a hand-written reverse pass through
the definitions above (including the dependence of layer 2 on h^1 of both endpoints).
Weights come in as one flat float32 blob, split in the order listed in ``_layout``; they
are promoted to float64 here.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .neighbors import pairs as _pairs

_CHUNK = 1 << 15


# --------------------------------------------------------------------------- parameters
@dataclass
class Model:
    kind: int                 # 0 = one interaction, 1 = two interactions with moments
    cutoff: float
    n_rbf: int
    width: int
    emb_dim: int
    n_species: int
    energy_scale: float
    w: dict                   # name -> float64 array

    @property
    def receptive_field(self) -> float:
        return self.cutoff * (1 if self.kind == 0 else 2)


def _layout(kind: int, K: int, F: int, D: int, Z: int):
    if kind == 0:
        return [("emb", (Z, D)), ("W_pair", (F, K + 2 * D)), ("W_atom1", (F, F)),
                ("w_atom2", (F,))]
    Q = 3 * F
    return [("emb", (Z, D)), ("W_pair1", (F, K + 2 * D)), ("U1", (F, Q)),
            ("W_pair2", (F, K + 2 * F)), ("U2", (F, Q)), ("W_out1", (F, F)),
            ("w_out2", (F,))]


def make_model(kind: int, cutoff: float, n_rbf: int, width: int, flat_weights,
               emb_dim: int = 16, n_species: int = 5, energy_scale: float = 0.01) -> Model:
    flat = np.asarray(flat_weights).astype(np.float64).ravel()
    w, o = {}, 0
    for name, shape in _layout(kind, n_rbf, width, emb_dim, n_species):
        n = int(np.prod(shape))
        w[name] = flat[o:o + n].reshape(shape).copy()
        o += n
    if o != flat.size:
        raise ValueError(f"weight blob has {flat.size} entries, model needs {o}")
    return Model(kind, float(cutoff), int(n_rbf), int(width), int(emb_dim), int(n_species),
                 float(energy_scale), w)


# --------------------------------------------------------------------------- pieces
def rbf(r: np.ndarray, cutoff: float, K: int):
    """Gaussian radial basis b_k(r) and its derivative db_k/dr, shape (P, K)."""
    mu = np.arange(K) * (cutoff / (K - 1))
    sigma = cutoff / (K - 1)
    x = r[:, None] - mu[None, :]
    b = np.exp(-(x * x) / (2.0 * sigma * sigma))
    db = -x / (sigma * sigma) * b
    return b, db


def cosine_cutoff(r: np.ndarray, cutoff: float):
    """f_c(r) = (cos(pi r/r_c) + 1)/2 inside the cutoff, 0 outside; and df_c/dr."""
    inside = r < cutoff
    fc = np.where(inside, 0.5 * (np.cos(np.pi * r / cutoff) + 1.0), 0.0)
    dfc = np.where(inside, -0.5 * np.pi / cutoff * np.sin(np.pi * r / cutoff), 0.0)
    return fc, dfc


def silu(t: np.ndarray) -> np.ndarray:
    return t / (1.0 + np.exp(-t))


def dsilu(t: np.ndarray) -> np.ndarray:
    s = 1.0 / (1.0 + np.exp(-t))
    return s * (1.0 + t * (1.0 - s))


def second_moment(u: np.ndarray) -> np.ndarray:
    """Traceless Y2(u) = u u^T - |u|^2 I/3, shape (P, 3, 3)."""
    uu = u[:, :, None] * u[:, None, :]
    tr = np.einsum("pa,pa->p", u, u)
    return uu - (tr / 3.0)[:, None, None] * np.eye(3)[None]


# --------------------------------------------------------------------------- helpers
def _system_sums(E_atom: np.ndarray, n_atoms: int, sys_offsets) -> np.ndarray:
    if sys_offsets is None:
        return np.array([E_atom.sum()])
    offs = np.asarray(sys_offsets, dtype=np.int64)
    return np.array([E_atom[a:b].sum() for a, b in zip(offs[:-1], offs[1:])])


def _pair_geometry(model: Model, d: np.ndarray):
    r = np.sqrt(np.einsum("pk,pk->p", d, d))
    b, db = rbf(r, model.cutoff, model.n_rbf)
    fc, dfc = cosine_cutoff(r, model.cutoff)
    return r, b, db, fc, dfc


def _accumulate_position_grad(dEdx: np.ndarray, i, j, dEdd: np.ndarray) -> None:
    """d_ij = x_j - x_i, so dE/dx_j += dE/dd_ij and dE/dx_i -= dE/dd_ij."""
    np.add.at(dEdx, j, dEdd)
    np.add.at(dEdx, i, -dEdd)


# --------------------------------------------------------------------------- kind 0
def _small(model: Model, pos, species, i, j, d):
    n = pos.shape[0]
    w = model.w
    F_w = model.width
    emb = w["emb"]
    # forward: pair messages summed on the receiver
    h = np.zeros((n, F_w))
    for s in range(0, len(i), _CHUNK):
        sl = slice(s, s + _CHUNK)
        r, b, _, fc, _ = _pair_geometry(model, d[sl])
        feat = np.concatenate([b, emb[species[i[sl]]], emb[species[j[sl]]]], axis=1)
        a = feat @ w["W_pair"].T
        m = fc[:, None] * silu(a)
        np.add.at(h, i[sl], m)
    # atom readout
    z = h @ w["W_atom1"].T
    E_atom = model.energy_scale * (silu(z) @ w["w_atom2"])
    # reverse pass: dE/dh_i
    dz = model.energy_scale * w["w_atom2"][None, :] * dsilu(z)
    dh = dz @ w["W_atom1"]
    dEdx = np.zeros((n, 3))
    K = model.n_rbf
    for s in range(0, len(i), _CHUNK):
        sl = slice(s, s + _CHUNK)
        r, b, db, fc, dfc = _pair_geometry(model, d[sl])
        feat = np.concatenate([b, emb[species[i[sl]]], emb[species[j[sl]]]], axis=1)
        a = feat @ w["W_pair"].T
        dm = dh[i[sl]]
        dfc_term = np.einsum("pc,pc->p", dm, silu(a))
        da = dm * fc[:, None] * dsilu(a)
        dfeat = da @ w["W_pair"]
        dr = dfc_term * dfc + np.einsum("pk,pk->p", dfeat[:, :K], db)
        _accumulate_position_grad(dEdx, i[sl], j[sl], (dr / r)[:, None] * d[sl])
    return E_atom, -dEdx


# --------------------------------------------------------------------------- kind 1
def _moments_layer(model: Model, Wp, src, i, j, d, n):
    """Forward of one interaction: returns M0 (n,F), M1 (n,F,3), M2 (n,F,3,3)."""
    F_w = model.width
    M0 = np.zeros((n, F_w))
    M1 = np.zeros((n, F_w, 3))
    M2 = np.zeros((n, F_w, 3, 3))
    for s in range(0, len(i), _CHUNK):
        sl = slice(s, s + _CHUNK)
        r, b, _, fc, _ = _pair_geometry(model, d[sl])
        feat = np.concatenate([b, src[i[sl]], src[j[sl]]], axis=1)
        a = feat @ Wp.T
        m = fc[:, None] * silu(a)
        u = d[sl] / model.cutoff
        Y2 = second_moment(u)
        np.add.at(M0, i[sl], m)
        np.add.at(M1, i[sl], m[:, :, None] * u[:, None, :])
        np.add.at(M2, i[sl], m[:, :, None, None] * Y2[:, None, :, :])
    return M0, M1, M2


def invariants(M0, M1, M2):
    """q = [M0 ; sum_a M1^2 ; sum_ab M2^2], channel-wise, shape (n, 3F)."""
    return np.concatenate([M0, np.einsum("ncA,ncA->nc", M1, M1),
                           np.einsum("ncab,ncab->nc", M2, M2)], axis=1)


def _moments_layer_backward(model: Model, Wp, src, i, j, d, dM0, dM1, dM2, dEdx, dsrc):
    """Reverse pass of one interaction.  Adds dE/dx into dEdx and, when dsrc is not None,
    dE/ds (receiver and sender feature blocks) into dsrc."""
    K = model.n_rbf
    S = src.shape[1]
    rc = model.cutoff
    for s in range(0, len(i), _CHUNK):
        sl = slice(s, s + _CHUNK)
        ii, jj, dd = i[sl], j[sl], d[sl]
        r, b, db, fc, dfc = _pair_geometry(model, dd)
        feat = np.concatenate([b, src[ii], src[jj]], axis=1)
        a = feat @ Wp.T
        sa = silu(a)
        m = fc[:, None] * sa
        u = dd / rc
        Y2 = second_moment(u)
        # dE/dm_ij (channel-wise) from the three moment sums of receiver i
        dm = (dM0[ii] + np.einsum("pca,pa->pc", dM1[ii], u)
              + np.einsum("pcab,pab->pc", dM2[ii], Y2))
        # dE/du through the angular factors u and Y2(u)
        G1 = np.einsum("pc,pca->pa", m, dM1[ii])
        G2 = np.einsum("pc,pcab->pab", m, dM2[ii])
        du = (G1 + np.einsum("pab,pb->pa", G2, u) + np.einsum("pba,pb->pa", G2, u)
              - (2.0 / 3.0) * np.einsum("paa->p", G2)[:, None] * u)
        # dE/da and the radial chain
        dfc_term = np.einsum("pc,pc->p", dm, sa)
        da = dm * fc[:, None] * dsilu(a)
        dfeat = da @ Wp
        dr = dfc_term * dfc + np.einsum("pk,pk->p", dfeat[:, :K], db)
        dEdd = (dr / r)[:, None] * dd + du / rc
        _accumulate_position_grad(dEdx, ii, jj, dEdd)
        if dsrc is not None:
            np.add.at(dsrc, ii, dfeat[:, K:K + S])
            np.add.at(dsrc, jj, dfeat[:, K + S:K + 2 * S])


def _invariants_backward(M0, M1, M2, dq, F_w):
    dM0 = dq[:, :F_w]
    dM1 = 2.0 * M1 * dq[:, F_w:2 * F_w, None]
    dM2 = 2.0 * M2 * dq[:, 2 * F_w:, None, None]
    return dM0, dM1, dM2


def _large(model: Model, pos, species, i, j, d):
    n = pos.shape[0]
    w = model.w
    F_w = model.width
    s1 = w["emb"][species]
    # interaction 1
    M0a, M1a, M2a = _moments_layer(model, w["W_pair1"], s1, i, j, d, n)
    q1 = invariants(M0a, M1a, M2a)
    z1 = q1 @ w["U1"].T
    h1 = silu(z1)
    # interaction 2 (senders and receivers carry h^1)
    M0b, M1b, M2b = _moments_layer(model, w["W_pair2"], h1, i, j, d, n)
    q2 = invariants(M0b, M1b, M2b)
    z2 = q2 @ w["U2"].T
    h2 = h1 + silu(z2)
    # readout
    y = h2 @ w["W_out1"].T
    E_atom = model.energy_scale * (silu(y) @ w["w_out2"])
    # reverse pass
    dy = model.energy_scale * w["w_out2"][None, :] * dsilu(y)
    dh2 = dy @ w["W_out1"]
    dz2 = dh2 * dsilu(z2)
    dq2 = dz2 @ w["U2"]
    dh1 = dh2.copy()
    dEdx = np.zeros((n, 3))
    _moments_layer_backward(model, w["W_pair2"], h1, i, j, d,
                            *_invariants_backward(M0b, M1b, M2b, dq2, F_w), dEdx, dh1)
    dz1 = dh1 * dsilu(z1)
    dq1 = dz1 @ w["U1"]
    _moments_layer_backward(model, w["W_pair1"], s1, i, j, d,
                            *_invariants_backward(M0a, M1a, M2a, dq1, F_w), dEdx, None)
    return E_atom, -dEdx


# --------------------------------------------------------------------------- public
def energy_forces(model: Model, pos, species, box: float, sys_offsets=None, pair_set=None):
    """Energy per system (FP64, shape (n_sys,)), forces (N, 3) in eV/A and per-atom
    energies (N,).  ``pair_set`` = (i, j, d) may be passed to skip the neighbor search."""
    pos = np.asarray(pos, dtype=np.float64)
    species = np.asarray(species, dtype=np.int64)
    if pair_set is None:
        pair_set = _pairs(pos, box, model.cutoff, sys_offsets)
    i, j, d = pair_set
    if model.kind == 0:
        E_atom, F = _small(model, pos, species, i, j, d)
    else:
        E_atom, F = _large(model, pos, species, i, j, d)
    return _system_sums(E_atom, pos.shape[0], sys_offsets), F, E_atom


def readout_magnitude(model: Model, pos, species, box: float, sys_offsets=None) -> np.ndarray:
    """Per-atom s_E sum_c |w_c SiLU(z_c)|: the size of the terms the readout adds up to
    E_i = s_E sum_c w_c SiLU(z_c) (z = W_atom1 h for the fast model, W_out1 h^2 for the
    reference model).  Rounding the readout's operands to a precision u moves E_i by a
    multiple of u times this, whatever the cancellation in E_i itself."""
    pos = np.asarray(pos, dtype=np.float64)
    species = np.asarray(species, dtype=np.int64)
    i, j, d = _pairs(pos, box, model.cutoff, sys_offsets)
    w = model.w
    n = pos.shape[0]
    if model.kind == 0:
        h = np.zeros((n, model.width))
        for s in range(0, len(i), _CHUNK):
            sl = slice(s, s + _CHUNK)
            _, b, _, fc, _ = _pair_geometry(model, d[sl])
            feat = np.concatenate([b, w["emb"][species[i[sl]]], w["emb"][species[j[sl]]]], axis=1)
            np.add.at(h, i[sl], fc[:, None] * silu(feat @ w["W_pair"].T))
        z, wo = h @ w["W_atom1"].T, w["w_atom2"]
    else:
        s1 = w["emb"][species]
        h1 = silu(invariants(*_moments_layer(model, w["W_pair1"], s1, i, j, d, n)) @ w["U1"].T)
        q2 = invariants(*_moments_layer(model, w["W_pair2"], h1, i, j, d, n))
        z, wo = (h1 + silu(q2 @ w["U2"].T)) @ w["W_out1"].T, w["w_out2"]
    return model.energy_scale * (np.abs(silu(z)) @ np.abs(wo))


def large_layer1_invariants(model: Model, pos, species, box: float, sys_offsets=None):
    """q^1 of the two-interaction model (exposed for the closed-form angular checks)."""
    pos = np.asarray(pos, dtype=np.float64)
    i, j, d = _pairs(pos, box, model.cutoff, sys_offsets)
    s1 = model.w["emb"][np.asarray(species)]
    return invariants(*_moments_layer(model, model.w["W_pair1"], s1, i, j, d, pos.shape[0]))


def force_error(F: np.ndarray, F_ref: np.ndarray) -> float:
    """Relative force RMSE ||F - F*||_2 / ||F*||_2 over all 3N components."""
    return float(np.linalg.norm(np.asarray(F, np.float64) - F_ref) / np.linalg.norm(F_ref))
