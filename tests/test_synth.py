"""Input generators: determinism and the shapes the workloads call for."""

import numpy as np

from oracle import neighbors as NB
from paper_2510_06562_amd import synth


def test_generators_are_deterministic():
    a, b = synth.water_4500(), synth.water_4500()
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.species, b.species)
    assert np.array_equal(synth.model_weights(synth.LARGE, 102), synth.model_weights(synth.LARGE, 102))
    m1, m2 = synth.molecule_batch(8, 3), synth.molecule_batch(8, 3)
    assert np.array_equal(m1.pos, m2.pos)


def test_water_geometry():
    sy = synth.water_box(27, 9.3, seed=5, jitter=0.0)
    o, h1, h2 = sy.pos[0::3], sy.pos[1::3], sy.pos[2::3]
    np.testing.assert_allclose(np.linalg.norm(h1 - o, axis=1), 0.96, rtol=1e-12)
    cosang = np.einsum("ij,ij->i", h1 - o, h2 - o) / 0.96**2
    np.testing.assert_allclose(np.degrees(np.arccos(cosang)), 104.5, rtol=1e-10)
    assert sy.n_atoms == 81


def test_workload_sizes():
    assert synth.water_192().n_atoms == 192
    assert synth.water_4500().n_atoms == 4500
    b = synth.molecule_batch(256, 3)
    sizes = np.diff(b.sys_offsets)
    assert b.n_sys == 256 and sizes.min() >= 20 and sizes.max() <= 120
    assert abs(b.n_atoms - 17920) < 1200


def test_batch_chains_are_self_avoiding():
    b = synth.molecule_batch(4, 9)
    for m in range(4):
        p = b.pos[b.sys_offsets[m]:b.sys_offsets[m + 1]]
        bonds = np.linalg.norm(np.diff(p, axis=0), axis=1)
        assert bonds.min() >= 1.1 - 1e-12 and bonds.max() <= 1.5 + 1e-12
        i, j, _ = NB.pairs_bruteforce(p, 0.0, 1.1 - 1e-9)
        assert np.all(np.abs(i - j) == 1) or len(i) == 0


def test_weight_blob_sizes_and_scale():
    ws = synth.model_weights(synth.SMALL, 101)
    wl = synth.model_weights(synth.LARGE, 102)
    assert ws.dtype == np.float32 and ws.size == 80 + 64 * 48 + 64 * 64 + 64
    assert wl.size == 80 + 128 * 64 + 128 * 384 + 128 * 288 + 128 * 384 + 128 * 128 + 128
    u = synth.unpack_weights(synth.LARGE, wl)
    assert abs(u["U1"].std() * np.sqrt(384) - 1.0) < 0.02


def test_hmr_masses():
    """Hydrogen mass repartitioning keeps every molecule's mass: in water each H gets
    3.024 amu and its oxygen 15.999 - 2 (3.024 - 1.008); in the random batch molecules
    no heavy atom ends lighter than the repartitioned hydrogens."""
    w = synth.water_192()
    m = w.hmr_masses()
    assert np.allclose(m[w.species == synth.H], 3.024)
    assert np.allclose(m[w.species == synth.O], 15.999 - 2 * (3.024 - 1.008))
    assert abs(m.sum() - w.masses().sum()) < 1e-9
    b = synth.molecule_batch(16, seed=3)
    mb = b.hmr_masses()
    for a, c in zip(b.sys_offsets[:-1], b.sys_offsets[1:]):
        assert abs(mb[a:c].sum() - b.masses()[a:c].sum()) < 1e-9
    heavy = b.species != synth.H
    assert mb[heavy].min() >= 3.024 - 1e-12
    assert mb[~heavy].min() >= synth.MASSES[synth.H] - 1e-12
    assert mb[~heavy].max() <= 3.024 + 1e-12


def test_maxwell_boltzmann_with_atom_masses():
    """Velocities drawn for per-atom masses have k_B T / m_i variance per component (the
    same normals scaled by sqrt(m_species / m_i)) and zero total momentum."""
    w = synth.water_4500()
    m = w.hmr_masses()
    v = synth.maxwell_boltzmann(w.species, 300.0, 5, masses=m)
    v0 = synth.maxwell_boltzmann(w.species, 300.0, 5)
    assert np.allclose((m[:, None] * v).sum(0), 0.0, atol=1e-9)
    # before the centre-of-mass shift the two draws differ by the per-atom scale only
    ratio = (v - v.mean(0)) / (v0 - v0.mean(0))
    h = w.species == synth.H
    assert abs(np.median(ratio[h]) - np.sqrt(1.008 / 3.024)) < 1e-3
    kT_over_m = (8.617333262e-5 * 300.0) * (1.602176634e-19 / 1.66053906660e-27 * 1e-10) / m
    assert abs(np.mean(v[h] ** 2 / kT_over_m[h, None]) - 1.0) < 0.05
