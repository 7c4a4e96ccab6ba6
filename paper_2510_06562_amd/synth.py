"""Seeded synthetic inputs: molecular systems, model weights and initial velocities.

This module is shared by the tests, the benchmark and the CPU oracle's checks.  It holds
none of the method's arithmetic (no neighbor search, no model, no integrator): only the
recipes that place atoms, draw weights and draw velocities.  Every array it returns is a
plain NumPy array, fully determined by the seed.

Layouts used throughout the project:
  * positions, velocities: float64, shape (N, 3) here (the device library stores the
    transposed structure-of-arrays form [3][N]);
  * species: int32 codes H=0, C=1, N=2, O=3, S=4;
  * box: cubic edge length L in Angstrom, 0.0 for open boundaries;
  * sys_offsets: int32 (n_sys + 1,) CSR offsets of independent molecules (batched form).

Units: Angstrom, femtosecond, atomic mass unit, electron-volt.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

H, C, N, O, S = 0, 1, 2, 3, 4
N_SPECIES = 5
SPECIES_NAMES = ("H", "C", "N", "O", "S")

# Conventional standard atomic weights (IUPAC abridged values), amu.  These are inputs of
# a simulation, not part of the method.
MASSES = np.array([1.008, 12.011, 14.007, 15.999, 32.06], dtype=np.float64)

# Used only to draw Maxwell-Boltzmann velocities (k_B T / m in Angstrom^2/fs^2).
_EV_PER_K = 8.617333262e-5          # Boltzmann constant, eV/K (CODATA 2018, exact)
# 1 eV/(amu*Angstrom^2) expressed in 1/fs^2, from the CODATA 2018 elementary charge and
# atomic mass constant.
_ANG_FS2_PER_EV_AMU = 1.602176634e-19 / 1.66053906660e-27 * 1e-30 * 1e20

# Water geometry.
_OH = 0.96
_HOH_DEG = 104.5


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class System:
    """A molecular configuration."""

    pos: np.ndarray                 # (N, 3) float64
    species: np.ndarray             # (N,) int32
    box: float                      # cubic edge, 0.0 = open
    sys_offsets: np.ndarray = field(default=None)  # (n_sys+1,) int32 or None
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_sys(self) -> int:
        return 1 if self.sys_offsets is None else int(len(self.sys_offsets) - 1)

    def masses(self) -> np.ndarray:
        return MASSES[self.species]

    def hmr_masses(self, h_mass: float = 3.024) -> np.ndarray:
        """Hydrogen mass repartitioning: every hydrogen gets h_mass (default three times
        its mass) and the difference is taken from its nearest heavy atom (minimum image;
        in a batch, within its molecule), so each molecule keeps its total mass.  A heavy
        atom gives at most what keeps it at h_mass (random synthetic molecules can put many
        hydrogens next to one atom); its hydrogens then share that amount equally."""
        from scipy.spatial import cKDTree
        m = self.masses().copy()
        offs = self.sys_offsets if self.sys_offsets is not None else np.array([0, self.n_atoms])
        for a, b in zip(offs[:-1], offs[1:]):
            sp = self.species[a:b]
            hyd = np.nonzero(sp == H)[0]
            heavy = np.nonzero(sp != H)[0]
            if len(hyd) == 0 or len(heavy) == 0:
                continue
            pos = self.pos[a:b]
            if self.box > 0.0:
                tree = cKDTree(np.mod(pos[heavy], self.box), boxsize=self.box)
                _, k = tree.query(np.mod(pos[hyd], self.box))
            else:
                _, k = cKDTree(pos[heavy]).query(pos[hyd])
            cnt = np.bincount(k, minlength=len(heavy))
            room = np.maximum(m[a + heavy] - h_mass, 0.0)
            dm = np.minimum(h_mass - MASSES[H], room / np.maximum(cnt, 1))
            m[a + hyd] = MASSES[H] + dm[k]
            m[a + heavy] -= cnt * dm
        return m


# --------------------------------------------------------------------------- rotations
def _haar_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed rotation matrices from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_rotation(seed: int) -> np.ndarray:
    return _haar_rotations(_rng(seed), 1)[0]


def _water_template() -> np.ndarray:
    half = math.radians(_HOH_DEG) / 2.0
    return np.array([
        [0.0, 0.0, 0.0],
        [_OH * math.sin(half), _OH * math.cos(half), 0.0],
        [-_OH * math.sin(half), _OH * math.cos(half), 0.0],
    ])


# --------------------------------------------------------------------------- water boxes
def water_box(n_mol: int, box: float, seed: int, jitter: float = 0.05) -> System:
    """Water molecules on a cubic lattice in a periodic box.

    The lattice has n_side = ceil(n_mol^(1/3)) sites per edge with spacing box/n_side and
    site centres at (i + 1/2) * spacing.  When n_mol is smaller than n_side^3 a seeded
    subset of sites is kept, in lattice order.  Each molecule (O, H, H with O-H 0.96 A,
    H-O-H 104.5 deg) gets a Haar-random orientation about its oxygen at the site centre;
    every atom is then jittered by N(0, jitter^2) per component.
    """
    rng = _rng(seed)
    n_side = int(math.ceil(round(n_mol ** (1.0 / 3.0), 9)))
    while n_side ** 3 < n_mol:
        n_side += 1
    a = box / n_side
    n_sites = n_side ** 3
    if n_mol < n_sites:
        sites = np.sort(rng.choice(n_sites, size=n_mol, replace=False))
    else:
        sites = np.arange(n_sites)
    ix = sites // (n_side * n_side)
    iy = (sites // n_side) % n_side
    iz = sites % n_side
    centres = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    R = _haar_rotations(rng, n_mol)
    tmpl = _water_template()
    pos = centres[:, None, :] + np.einsum("mab,kb->mka", R, tmpl)
    pos = pos.reshape(-1, 3)
    pos = pos + rng.standard_normal(pos.shape) * jitter
    species = np.tile(np.array([O, H, H], dtype=np.int32), n_mol)
    return System(pos=np.ascontiguousarray(pos), species=species, box=float(box),
                  name=f"water{n_mol}")


def water_192(seed: int = 0) -> System:
    """64 H2O (192 atoms) in a 12.42 A periodic cube on a 4x4x4 lattice."""
    return water_box(64, 12.42, seed)


def water_4500(seed: int = 1) -> System:
    """1,500 H2O (4,500 atoms) in a 35.5 A periodic cube; 1,500 of 12^3 sites."""
    return water_box(1500, 35.5, seed)


# --------------------------------------------------------------------------- chains
_ORGANIC_P = np.array([0.50, 0.30, 0.08, 0.10, 0.02])
_PROTEIN_P = np.array([0.49, 0.32, 0.08, 0.10, 0.01])


def _random_unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _open_chain(rng: np.random.Generator, n: int, bond_lo: float, bond_hi: float,
                min_nb: float) -> np.ndarray:
    """Self-avoiding random walk: each new atom sits a U[bond_lo, bond_hi] bond away from
    the previous one and at least min_nb from every other placed atom."""
    while True:
        pos = np.zeros((n, 3))
        ok = True
        for k in range(1, n):
            placed = False
            for _ in range(1000):
                cand = pos[k - 1] + rng.uniform(bond_lo, bond_hi) * _random_unit(rng)
                if k >= 2:
                    dmin = np.min(np.linalg.norm(pos[: k - 1] - cand, axis=1))
                    if dmin < min_nb:
                        continue
                pos[k] = cand
                placed = True
                break
            if not placed:
                ok = False
                break
        if ok:
            return pos - pos.mean(axis=0)


def molecule_batch(n_mol: int = 256, seed: int = 3, lo: int = 10, hi: int = 60) -> System:
    """Independent open molecules for the batched form.

    Each molecule draws n ~ U{lo..hi} and holds 2n atoms (so the expected total is
    n_mol * (lo + hi) = 17,920 for the default 256 molecules).  Elements are i.i.d. with
    H:C:N:O:S = 0.50:0.30:0.08:0.10:0.02; atoms are placed as a self-avoiding chain with
    1.1-1.5 A bonds, centred on its centroid.  Every molecule keeps its own coordinates
    (they overlap in space; pairs never cross molecules).
    """
    rng = _rng(seed)
    sizes = 2 * rng.integers(lo, hi + 1, size=n_mol)
    pos_list, sp_list = [], []
    for n in sizes:
        sp_list.append(rng.choice(N_SPECIES, size=int(n), p=_ORGANIC_P).astype(np.int32))
        pos_list.append(_open_chain(rng, int(n), 1.1, 1.5, 1.1))
    offs = np.zeros(n_mol + 1, dtype=np.int32)
    offs[1:] = np.cumsum(sizes)
    return System(pos=np.ascontiguousarray(np.concatenate(pos_list)),
                  species=np.concatenate(sp_list), box=0.0, sys_offsets=offs,
                  name=f"batch{n_mol}")


def _minimage(d: np.ndarray, box: float) -> np.ndarray:
    return d - box * np.rint(d / box)


def solvated_chain(seed: int = 4, box: float = 100.0, n_chain: int = 5000,
                   n_water: int = 31667, n_side: int = 33) -> System:
    """A protein-shaped system: a periodic random-walk chain of n_chain atoms (C 32%,
    N 8%, O 10%, S 1%, H 49%; 1.0-1.5 A bonds; non-bonded distance >= 1.5 A) in a cube
    filled with waters on an n_side^3 lattice.  Sites whose oxygen lies within 2.0 A of a
    chain atom are dropped and a seeded n_water of the rest are kept.  With the defaults
    N = 5,000 + 3 * 31,667 = 100,001 atoms."""
    rng = _rng(seed)
    chain = np.zeros((n_chain, 3))
    chain[0] = rng.uniform(0, box, 3)
    # coarse cell hash for the self-avoidance test
    cell = 3.0
    nc = int(box // cell)
    grid: dict = {}

    def key(p):
        c = np.floor((p % box) / (box / nc)).astype(int) % nc
        return int(c[0]), int(c[1]), int(c[2])

    def near(p, skip):
        kx, ky, kz = key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for idx in grid.get(((kx + dx) % nc, (ky + dy) % nc, (kz + dz) % nc), ()):
                        if idx == skip:
                            continue
                        if np.linalg.norm(_minimage(chain[idx] - p, box)) < 1.5:
                            return True
        return False

    grid.setdefault(key(chain[0]), []).append(0)
    for k in range(1, n_chain):
        for _ in range(1000):
            cand = chain[k - 1] + rng.uniform(1.0, 1.5) * _random_unit(rng)
            if not near(cand, k - 1):
                break
        chain[k] = cand % box
        grid.setdefault(key(chain[k]), []).append(k)
    chain_sp = rng.choice(N_SPECIES, size=n_chain, p=_PROTEIN_P).astype(np.int32)

    a = box / n_side
    idx = np.arange(n_side ** 3)
    centres = (np.stack([idx // (n_side * n_side), (idx // n_side) % n_side, idx % n_side],
                        axis=1) + 0.5) * a
    keep = np.ones(len(centres), dtype=bool)
    for s in range(0, len(centres), 4096):
        d = _minimage(centres[s:s + 4096, None, :] - chain[None, :, :], box)
        keep[s:s + 4096] = np.min(np.einsum("abk,abk->ab", d, d), axis=1) >= 4.0
    free = np.nonzero(keep)[0]
    if len(free) < n_water:
        raise ValueError(f"only {len(free)} water sites free, {n_water} requested")
    sites = np.sort(rng.choice(free, size=n_water, replace=False))
    R = _haar_rotations(rng, n_water)
    wpos = centres[sites][:, None, :] + np.einsum("mab,kb->mka", R, _water_template())
    wpos = wpos.reshape(-1, 3)
    wpos = wpos + rng.standard_normal(wpos.shape) * 0.05
    pos = np.concatenate([chain, wpos]) % box
    species = np.concatenate([chain_sp, np.tile(np.array([O, H, H], dtype=np.int32), n_water)])
    return System(pos=np.ascontiguousarray(pos), species=species, box=float(box),
                  name="solvated100k")


# --------------------------------------------------------------------------- models
@dataclass(frozen=True)
class ModelSpec:
    """Hyper-parameters of one synthetic potential.

    kind 0 = one-interaction model (receiver/sender species embedding, summed pair
    messages, 2-layer atom readout); kind 1 = two-interaction model with l <= 2 Cartesian
    moments, a residual second interaction and a 2-layer readout.
    """

    kind: int
    cutoff: float
    n_rbf: int
    width: int
    emb_dim: int = 16
    n_species: int = N_SPECIES
    energy_scale: float = 0.01
    n_moments: int = 10  # only for kind 1: 1 + 3 + 6 stored components (see shapes)

    def shapes(self):
        """(name, shape, fan_in) in drawing and packing order."""
        K, F, D, Z = self.n_rbf, self.width, self.emb_dim, self.n_species
        if self.kind == 0:
            return [("emb", (Z, D), Z), ("W_pair", (F, K + 2 * D), K + 2 * D),
                    ("W_atom1", (F, F), F), ("w_atom2", (F,), F)]
        Q = 3 * F
        return [("emb", (Z, D), Z), ("W_pair1", (F, K + 2 * D), K + 2 * D),
                ("U1", (F, Q), Q), ("W_pair2", (F, K + 2 * F), K + 2 * F),
                ("U2", (F, Q), Q), ("W_out1", (F, F), F), ("w_out2", (F,), F)]

    def n_weights(self) -> int:
        return int(sum(int(np.prod(s)) for _, s, _ in self.shapes()))


SMALL = ModelSpec(kind=0, cutoff=3.5, n_rbf=16, width=64)
LARGE = ModelSpec(kind=1, cutoff=5.2, n_rbf=32, width=128)
# the message-passing fast model (two interactions, as the reference model) at the fast
# model's cutoff
SMALL_MP = ModelSpec(kind=1, cutoff=3.5, n_rbf=32, width=128)
SMALL_SEED = 101
LARGE_SEED = 102
SMALL_MP_SEED = 103


def model_weights(spec: ModelSpec, seed: int) -> np.ndarray:
    """Flat float32 weight blob: every entry i.i.d. N(0, 1/fan_in), drawn row-major in
    the order of ``spec.shapes()`` from PCG64(seed), then rounded to float32."""
    rng = _rng(seed)
    parts = []
    for _, shape, fan_in in spec.shapes():
        parts.append((rng.standard_normal(shape) / math.sqrt(fan_in)).ravel())
    return np.concatenate(parts).astype(np.float32)


def unpack_weights(spec: ModelSpec, flat: np.ndarray) -> dict:
    """Split a flat blob into named arrays (views, dtype preserved)."""
    out, o = {}, 0
    for name, shape, _ in spec.shapes():
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    if o != flat.size:
        raise ValueError(f"weight blob has {flat.size} entries, spec needs {o}")
    return out


# --------------------------------------------------------------------------- velocities
def maxwell_boltzmann(species: np.ndarray, T: float, seed: int,
                      sys_offsets: np.ndarray | None = None,
                      masses: np.ndarray | None = None) -> np.ndarray:
    """v ~ N(0, k_B T / m) per component in A/fs, centre-of-mass velocity removed (per
    molecule when sys_offsets is given), not rescaled.  m: the species masses, or the
    per-atom `masses` when given (e.g. repartitioned)."""
    rng = _rng(seed)
    m = MASSES[species] if masses is None else np.asarray(masses, dtype=np.float64)
    sd = np.sqrt(_EV_PER_K * T * _ANG_FS2_PER_EV_AMU / m)
    v = rng.standard_normal((len(species), 3)) * sd[:, None]
    offs = np.array([0, len(species)]) if sys_offsets is None else sys_offsets
    for a, b in zip(offs[:-1], offs[1:]):
        if b > a:
            v[a:b] -= (m[a:b, None] * v[a:b]).sum(0) / m[a:b].sum()
    return v


# --------------------------------------------------------------------------- workloads
WORKLOADS = {
    "water192": dict(system=lambda: water_192(0), vel_seed=200),
    "water4500": dict(system=lambda: water_4500(1), vel_seed=201),
    "batch256": dict(system=lambda: molecule_batch(256, 3), vel_seed=203),
    "solvated100k": dict(system=lambda: solvated_chain(4), vel_seed=204),
}
