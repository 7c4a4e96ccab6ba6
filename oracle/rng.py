"""Counter-based normal deviates for the Langevin O-step (oracle; test infrastructure only).

The thermostat of Algorithm 1 (its O-step, exact Ornstein-Uhlenbeck update of the
velocities) draws one standard normal per velocity component.  So that the HIP path and
this oracle use the same numbers without passing them around, both implement the same
counter-based generator from its published definition: Philox4x32 with 10 rounds
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).

Philox4x32 round, counter (c0, c1, c2, c3), key (k0, k1):
    (hi0, lo0) = 32x32 -> 64-bit product of 0xD2511F53 and c0
    (hi1, lo1) = 32x32 -> 64-bit product of 0xCD9E8D57 and c2
    next counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
The first round uses the key as given; before each further round the key is bumped by
the Weyl constants (0x9E3779B9, 0xBB67AE85), modulo 2^32.

Mapping to normals (the convention shared with the HIP path):
  * the k-th O-step of a state (k = 0, 1, ...) draws, for atom i, the 4 words
    r = Philox4x32-10(counter = (i, k mod 2^32, k div 2^32, 0), key = (seed mod 2^32,
    seed div 2^32));
  * u_j = (r_j + 1/2) / 2^32 in float64, so 0 < u_j < 1;
  * Box-Muller: xi_x = sqrt(-2 ln u_0) cos(2 pi u_1), xi_y = sqrt(-2 ln u_0) sin(2 pi u_1),
    xi_z = sqrt(-2 ln u_2) cos(2 pi u_3).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
TWO_PI = 2.0 * np.pi


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: array [..., 4] of uint32 words, key: [..., 2].
    Returns the [..., 4] uint32 output words (as uint64 arrays holding 32-bit values)."""
    c = [np.asarray(ctr[..., j], dtype=np.uint64) & MASK32 for j in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c[0]            # < 2^64: exact in uint64
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def o_step_normals(n_atoms: int, k: int, seed: int) -> np.ndarray:
    """Standard normals xi [n_atoms, 3] of the k-th O-step (see the module docstring)."""
    i = np.arange(n_atoms, dtype=np.uint64)
    ctr = np.zeros((n_atoms, 4), dtype=np.uint64)
    ctr[:, 0] = i
    ctr[:, 1] = np.uint64(k & 0xFFFFFFFF)
    ctr[:, 2] = np.uint64((k >> 32) & 0xFFFFFFFF)
    key = np.zeros((n_atoms, 2), dtype=np.uint64)
    key[:, 0] = np.uint64(seed & 0xFFFFFFFF)
    key[:, 1] = np.uint64((seed >> 32) & 0xFFFFFFFF)
    r = philox4x32_10(ctr, key)
    u = (r.astype(np.float64) + 0.5) * 2.0 ** -32
    rad0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    rad2 = np.sqrt(-2.0 * np.log(u[:, 2]))
    xi = np.empty((n_atoms, 3))
    xi[:, 0] = rad0 * np.cos(TWO_PI * u[:, 1])
    xi[:, 1] = rad0 * np.sin(TWO_PI * u[:, 1])
    xi[:, 2] = rad2 * np.cos(TWO_PI * u[:, 3])
    return xi


class OStepNoise:
    """Thermostat hook for the oracle integrators: the O-step of Algorithm 1 with the
    normals of successive O-steps k0, k0 + 1, ... of one seed."""

    def __init__(self, m: np.ndarray, gamma: float, T: float, seed: int, k0: int = 0):
        from .integrators import langevin_o
        self._o = langevin_o
        self.m, self.gamma, self.T, self.seed, self.k = m, gamma, T, seed, k0

    def __call__(self, v: np.ndarray, h: float) -> np.ndarray:
        xi = o_step_normals(v.shape[0], self.k, self.seed)
        self.k += 1
        return self._o(v, self.m, h, self.gamma, self.T, xi)
