"""Integrators in FP64 (oracle; test infrastructure only).

Algorithm 1 of the paper (MTS integration step with force splitting) is followed step by
step: on the first call both forces are evaluated; the outer level applies half-kicks
with the slow force F - F_small; in between, n_slow inner steps of length dt/n_slow each
do a half-kick with F_small, a half-drift, the thermostat, a half-drift, a fresh F_small
and a half-kick; a fresh F closes the step.  Symbols follow the paper: x coordinates,
v velocities, dt the outer step, m masses, n_slow the number of inner steps.

The single-time-step baseline of the experiments (BAOAB Langevin at 1 fs with the
reference model) is ``sts_step``.  With zero friction the thermostat is the identity and
both reduce to velocity Verlet (the kick-drift-drift-kick form).

Units: x in A, v in A/fs, forces in eV/A, masses in amu, time in fs.  Newton's law then
reads dv/dt = KAPPA * F / m with KAPPA = 1 eV/(A amu) in A/fs^2.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

# 1 eV / (A * amu) in A / fs^2: elementary charge / atomic mass constant (CODATA 2018)
# times 1e-20 (m/s^2 -> A/fs^2) times 1e10 (per A instead of per m).
KAPPA = 1.602176634e-19 / (1.0e-10 * 1.66053906660e-27) * 1.0e-20
K_BOLTZMANN = 8.617333262e-5   # eV / K

ForceFn = Callable[[np.ndarray], tuple]   # x -> (energy, forces (N,3))


def kinetic_energy(v: np.ndarray, m: np.ndarray) -> float:
    """KE = sum_i m_i |v_i|^2 / 2 in eV."""
    return float(0.5 * np.sum(m[:, None] * v * v) / KAPPA)


def temperature(v: np.ndarray, m: np.ndarray) -> float:
    """Instantaneous temperature with 3N - 3 degrees of freedom."""
    n = v.shape[0]
    return 2.0 * kinetic_energy(v, m) / ((3 * n - 3) * K_BOLTZMANN)


def langevin_o(v: np.ndarray, m: np.ndarray, h: float, gamma: float, T: float,
               xi: np.ndarray) -> np.ndarray:
    """Exact Ornstein-Uhlenbeck update over time h (the O of BAOAB):
    v <- c v + sqrt((1 - c^2) k_B T KAPPA / m) xi, c = exp(-gamma h); xi ~ N(0, 1) is
    supplied by the caller.  Identity when gamma = 0."""
    if gamma == 0.0:
        return v
    c = np.exp(-gamma * h)
    sd = np.sqrt((1.0 - c * c) * K_BOLTZMANN * T * KAPPA / m)
    return c * v + sd[:, None] * xi


@dataclass
class MTSState:
    """Dynamic state carried between calls of Algorithm 1."""

    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    F: Optional[np.ndarray] = None          # reference-model forces at x
    F_small: Optional[np.ndarray] = None    # fast-model forces at x
    E: float = 0.0                           # reference-model energy at x
    E_small: float = 0.0
    first_step: bool = True
    n_small_evals: int = 0
    n_large_evals: int = 0
    history: list = field(default_factory=list)


def _kick(v, F, m, tau):
    """v <- v + tau/m * F (tau in fs, dv in A/fs)."""
    return v + (tau * KAPPA / m)[:, None] * F


def _drift(x, v, tau):
    return x + tau * v


def mts_step(st: MTSState, dt: float, n_slow: int, small: ForceFn, large: ForceFn,
             thermo: Optional[Callable[[np.ndarray, float], np.ndarray]] = None) -> MTSState:
    """One outer step of Algorithm 1 (BAOAB-RESPA with force splitting F - F_small)."""
    if thermo is None:
        thermo = lambda v, h: v  # noqa: E731  (gamma = 0)
    if st.first_step:
        st.E_small, st.F_small = small(st.x)
        st.E, st.F = large(st.x)
        st.n_small_evals += 1
        st.n_large_evals += 1
        st.first_step = False
    h = dt / n_slow
    st.v = _kick(st.v, st.F - st.F_small, st.m, dt / 2.0)
    for _ in range(n_slow):
        st.v = _kick(st.v, st.F_small, st.m, h / 2.0)
        st.x = _drift(st.x, st.v, h / 2.0)
        st.v = thermo(st.v, h)
        st.x = _drift(st.x, st.v, h / 2.0)
        st.E_small, st.F_small = small(st.x)
        st.n_small_evals += 1
        st.v = _kick(st.v, st.F_small, st.m, h / 2.0)
    st.E, st.F = large(st.x)
    st.n_large_evals += 1
    st.v = _kick(st.v, st.F - st.F_small, st.m, dt / 2.0)
    return st


def sts_step(st: MTSState, dt: float, force: ForceFn,
             thermo: Optional[Callable[[np.ndarray, float], np.ndarray]] = None) -> MTSState:
    """One single-time-step BAOAB step with one model (velocity Verlet when gamma = 0)."""
    if thermo is None:
        thermo = lambda v, h: v  # noqa: E731
    if st.first_step:
        st.E, st.F = force(st.x)
        st.n_large_evals += 1
        st.first_step = False
    st.v = _kick(st.v, st.F, st.m, dt / 2.0)
    st.x = _drift(st.x, st.v, dt / 2.0)
    st.v = thermo(st.v, dt)
    st.x = _drift(st.x, st.v, dt / 2.0)
    st.E, st.F = force(st.x)
    st.n_large_evals += 1
    st.v = _kick(st.v, st.F, st.m, dt / 2.0)
    return st


def conserved_energy(st: MTSState) -> float:
    """H = KE + E_reference (the quantity NVE dynamics conserves)."""
    return kinetic_energy(st.v, st.m) + st.E
