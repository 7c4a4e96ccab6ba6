"""Pair sets under the minimum-image convention (oracle; test infrastructure only).

The paper does not describe its neighbor search; the models only need, for each receiver
atom i, the set of sender atoms j != i closer than the cutoff.  This module computes that
set by its definition:

    d_ij = x_j - x_i - L * rint((x_j - x_i) / L)    (periodic cube of edge L)
    d_ij = x_j - x_i                                 (open boundaries, L = 0)
    N(i) = { j != i : |d_ij| < r_c }

With open boundaries and a batch of molecules (CSR ``sys_offsets``), j must belong to
the same molecule as i.  Pairs are returned sorted by (i, j).
"""

from __future__ import annotations

import numpy as np


def minimage(d: np.ndarray, box: float) -> np.ndarray:
    """Minimum-image displacement (identity for open boundaries)."""
    if box == 0.0:
        return d
    return d - box * np.rint(d / box)


def _check_box(box: float, cutoff: float) -> None:
    if box != 0.0 and not cutoff < 0.5 * box:
        raise ValueError(f"cutoff {cutoff} must be below half the box edge {box}")


def _molecule_of(n: int, sys_offsets) -> np.ndarray:
    if sys_offsets is None:
        return np.zeros(n, dtype=np.int64)
    offs = np.asarray(sys_offsets, dtype=np.int64)
    return np.repeat(np.arange(len(offs) - 1), np.diff(offs))


def pairs_bruteforce(pos: np.ndarray, box: float, cutoff: float, sys_offsets=None,
                     chunk: int = 256):
    """All ordered pairs within the cutoff by testing every (i, j).  Returns (i, j, d)
    with d = d_ij of shape (P, 3)."""
    _check_box(box, cutoff)
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    mol = _molecule_of(n, sys_offsets)
    I, J, D = [], [], []
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        d = minimage(pos[None, :, :] - pos[a:b, None, :], box)   # [i - a, j, 3]
        r2 = np.einsum("ijk,ijk->ij", d, d)
        mask = r2 < cutoff * cutoff
        mask[np.arange(b - a), np.arange(a, b)] = False
        mask &= mol[a:b, None] == mol[None, :]
        ii, jj = np.nonzero(mask)
        I.append(ii + a)
        J.append(jj)
        D.append(d[ii, jj])
    i = np.concatenate(I).astype(np.int64)
    j = np.concatenate(J).astype(np.int64)
    d = np.concatenate(D) if D else np.zeros((0, 3))
    return i, j, d


def pairs_kdtree(pos: np.ndarray, box: float, cutoff: float, sys_offsets=None):
    """Same set as ``pairs_bruteforce`` found with a periodic k-d tree (large boxes)."""
    from scipy.spatial import cKDTree

    _check_box(box, cutoff)
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    if box != 0.0:
        tree = cKDTree(np.mod(pos, box), boxsize=box)
    else:
        tree = cKDTree(pos)
    pr = tree.query_pairs(cutoff, output_type="ndarray")
    i = np.concatenate([pr[:, 0], pr[:, 1]]).astype(np.int64)
    j = np.concatenate([pr[:, 1], pr[:, 0]]).astype(np.int64)
    d = minimage(pos[j] - pos[i], box)
    keep = np.einsum("pk,pk->p", d, d) < cutoff * cutoff
    mol = _molecule_of(n, sys_offsets)
    keep &= mol[i] == mol[j]
    i, j, d = i[keep], j[keep], d[keep]
    order = np.lexsort((j, i))
    return i[order], j[order], d[order]


def pairs(pos: np.ndarray, box: float, cutoff: float, sys_offsets=None):
    """Dispatch: brute force for small systems, k-d tree otherwise."""
    n = np.asarray(pos).shape[0]
    if n <= 6000:
        return pairs_bruteforce(pos, box, cutoff, sys_offsets)
    return pairs_kdtree(pos, box, cutoff, sys_offsets)
