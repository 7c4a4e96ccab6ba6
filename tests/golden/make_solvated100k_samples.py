"""Writes solvated100k_samples.json: oracle per-atom energies and forces of sampled atoms of
the 100,001-atom solvated system, for the full-size GPU parity test.

Only the oracle (and the seeded input recipe) is used.  An atom's energy depends on the
atoms within n_int * r_c of it (its receptive field: one interaction of 3.5 A for the fast
model, two of 5.2 A for the reference model), and its force on the atoms within twice
that, so each value is computed exactly on the open cluster of atoms within that radius
(plus 0.5 A) around the sampled atom, with minimum-image coordinates relative to it.

Run from the repository root:  python tests/golden/make_solvated100k_samples.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import potentials as OP  # noqa: E402
from paper_2510_06562_amd import synth  # noqa: E402

RECEPTIVE = {"small": 3.5, "large": 10.4}
SPECS = {"small": (synth.SMALL, synth.SMALL_SEED), "large": (synth.LARGE, synth.LARGE_SEED)}


def samples(n, n_chain=5000):
    """Seeded atoms: half from the chain (the first n_chain atoms), half from the water."""
    rng = np.random.default_rng(2024)
    chain = rng.choice(n_chain, size=8, replace=False)
    water = n_chain + rng.choice(n - n_chain, size=8, replace=False)
    return np.sort(np.concatenate([chain, water])).tolist()


def cluster(sy, i, radius):
    d = sy.pos - sy.pos[i]
    d -= sy.box * np.rint(d / sy.box)
    r = np.linalg.norm(d, axis=1)
    sel = np.nonzero(r < radius)[0]
    sel = np.concatenate([[i], sel[sel != i]])
    return d[sel], sy.species[sel]


def main():
    sy = synth.solvated_chain()
    atoms = samples(sy.n_atoms)
    out = {"system": "solvated100k", "n_atoms": int(sy.n_atoms), "atoms": atoms,
           "energy": {}, "force": {}, "force_atoms": {}}
    for which in ("small", "large"):
        spec, seed = SPECS[which]
        w = synth.model_weights(spec, seed)
        m = OP.make_model(spec.kind, spec.cutoff, spec.n_rbf, spec.width, w,
                          energy_scale=spec.energy_scale)
        R = RECEPTIVE[which]
        out["energy"][which] = []
        for i in atoms:
            p, s = cluster(sy, i, R + 0.5)
            _, _, Ea = OP.energy_forces(m, p, s, 0.0)
            out["energy"][which].append(float(Ea[0]))
        # forces need twice the radius: every atom for the fast model, two (one chain, one
        # water) for the reference model, whose clusters hold ~4,000 atoms
        f_atoms = atoms if which == "small" else [atoms[0], atoms[-1]]
        out["force_atoms"][which] = f_atoms
        out["force"][which] = []
        for i in f_atoms:
            p, s = cluster(sy, i, 2 * R + 0.5)
            _, F, _ = OP.energy_forces(m, p, s, 0.0)
            out["force"][which].append([float(x) for x in F[0]])
    with open(os.path.join(HERE, "solvated100k_samples.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
