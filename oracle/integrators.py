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


def _max_force_difference(st: MTSState) -> float:
    """max_i |F_i - F_small,i| (eV/A) at the state's positions."""
    return float(np.max(np.linalg.norm(st.F - st.F_small, axis=1)))


def mts_step_monitored(st: MTSState, dt: float, n_slow: int, small: ForceFn, large: ForceFn,
                       threshold: float) -> tuple:
    """One outer step of Algorithm 1 guarded by the force-difference check of the paper's
    protein-ligand runs (Results: frames whose per-atom |F - F_small| exceeds an
    unphysical threshold, 150 kcal/mol/A, are integrated with single time steps instead).
    Reading used here: the outer step is taken as usual; if either of its two slow kicks
    sees an atom with |F - F_small| > threshold, the step is discarded and redone from its
    starting state as n_slow single-time-step steps of dt/n_slow with the reference model,
    after which both forces are evaluated afresh.  NVE only (no thermostat).
    Returns (state, worst, redone): worst is the largest |F - F_small| of the RESPA step's
    two kicks (kept or discarded), redone whether it was replaced."""
    start = MTSState(x=st.x.copy(), v=st.v.copy(), m=st.m,
                     F=None if st.F is None else st.F.copy(),
                     F_small=None if st.F_small is None else st.F_small.copy(),
                     E=st.E, E_small=st.E_small, first_step=st.first_step)
    trial = MTSState(x=st.x.copy(), v=st.v.copy(), m=st.m, F=start.F, F_small=start.F_small,
                     E=st.E, E_small=st.E_small, first_step=st.first_step)
    if trial.first_step:
        trial.E_small, trial.F_small = small(trial.x)
        trial.E, trial.F = large(trial.x)
        trial.first_step = False
    worst = _max_force_difference(trial)                      # the opening slow kick
    mts_step(trial, dt, n_slow, small, large)
    worst = max(worst, _max_force_difference(trial))          # the closing slow kick
    if worst <= threshold:
        return trial, worst, False
    redo = MTSState(x=start.x, v=start.v, m=st.m, first_step=True)
    for _ in range(n_slow):
        sts_step(redo, dt / n_slow, large)
    redo.first_step = True   # the next outer step evaluates both models afresh
    return redo, worst, True


def conserved_energy(st: MTSState) -> float:
    """H = KE + E_reference (the quantity NVE dynamics conserves)."""
    return kinetic_energy(st.v, st.m) + st.E
