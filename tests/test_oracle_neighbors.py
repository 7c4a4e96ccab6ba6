"""Pins of the oracle's pair set: brute force vs k-d tree, hand-worked periodic images,
batched molecules and the box-size guard."""

import numpy as np
import pytest

from oracle import neighbors as NB
from paper_2510_06562_amd import synth


def _as_set(i, j):
    return set(zip(i.tolist(), j.tolist()))


def test_periodic_image_by_hand():
    # two atoms 0.2 A apart through the x face of a 10 A box
    L = 10.0
    pos = np.array([[0.1, 5.0, 5.0], [9.9, 5.0, 5.0], [5.0, 5.0, 5.0]])
    i, j, d = NB.pairs_bruteforce(pos, L, 1.0)
    assert _as_set(i, j) == {(0, 1), (1, 0)}
    k = list(zip(i, j)).index((0, 1))
    np.testing.assert_allclose(d[k], [-0.2, 0.0, 0.0], atol=1e-12)
    # the same atoms in an open box are 9.8 A apart
    i, j, _ = NB.pairs_bruteforce(pos, 0.0, 1.0)
    assert len(i) == 0


def test_strict_cutoff_and_self_excluded():
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    assert len(NB.pairs_bruteforce(pos, 0.0, 1.0)[0]) == 0          # |d| = rc is outside
    i, j, _ = NB.pairs_bruteforce(pos, 0.0, 1.0 + 1e-9)
    assert _as_set(i, j) == {(0, 1), (1, 0)}


def test_cutoff_must_be_below_half_box():
    pos = np.zeros((2, 3))
    with pytest.raises(ValueError):
        NB.pairs_bruteforce(pos, 10.0, 5.0)


@pytest.mark.parametrize("cut", [3.5, 5.2])
def test_kdtree_matches_bruteforce_water(cut):
    sy = synth.water_192()
    a = NB.pairs_bruteforce(sy.pos, sy.box, cut)
    b = NB.pairs_kdtree(sy.pos, sy.box, cut)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_allclose(a[2], b[2], atol=1e-12)


def test_kdtree_matches_bruteforce_random_box_with_wrapped_coords():
    rng = np.random.default_rng(7)
    pos = rng.uniform(-20.0, 40.0, size=(1500, 3))    # far outside [0, L): minimage wraps
    a = NB.pairs_bruteforce(pos, 20.0, 5.2)
    b = NB.pairs_kdtree(pos, 20.0, 5.2)
    assert _as_set(*a[:2]) == _as_set(*b[:2])


def test_batched_molecules_do_not_interact():
    sy = synth.molecule_batch(6, seed=11)
    i, j, _ = NB.pairs_bruteforce(sy.pos, 0.0, 5.2, sy.sys_offsets)
    mol = np.repeat(np.arange(6), np.diff(sy.sys_offsets))
    assert np.all(mol[i] == mol[j])
    # every molecule alone gives the same pairs
    for m in range(6):
        a, b = sy.sys_offsets[m], sy.sys_offsets[m + 1]
        ii, jj, _ = NB.pairs_bruteforce(sy.pos[a:b], 0.0, 5.2)
        sel = (i >= a) & (i < b)
        assert _as_set(ii + a, jj + a) == _as_set(i[sel], j[sel])
    b = NB.pairs_kdtree(sy.pos, 0.0, 5.2, sy.sys_offsets)
    assert _as_set(i, j) == _as_set(*b[:2])


def test_pair_set_is_symmetric_and_sorted():
    sy = synth.water_192()
    i, j, d = NB.pairs(sy.pos, sy.box, 5.2)
    assert _as_set(i, j) == _as_set(j, i)
    key = i * 10_000 + j
    assert np.all(np.diff(key) > 0)
    # density check: liquid-like water (0.1 atoms/A^3) has ~4/3 pi rc^3 * 0.1 neighbors
    assert 14.0 < len(i) / 192 < 19.0 or 55.0 < len(i) / 192 < 65.0
