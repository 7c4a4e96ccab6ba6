"""Shared helpers of the GPU tests: seeded systems, the two synthetic models, the oracle's
reference values (computed once per session) and the device wrappers."""

import functools
import sys

import numpy as np

from oracle import integrators as OI
from oracle import neighbors as ON
from oracle import potentials as OP
from paper_2510_06562_amd import synth


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def system(name):
    if name == "water192":
        return synth.water_192()
    if name == "water4500":
        return synth.water_4500()
    if name == "batch16":
        return synth.molecule_batch(16, seed=3)
    if name == "batch256":
        return synth.molecule_batch(256, seed=3)
    if name == "open60":
        b = synth.molecule_batch(1, seed=12, lo=30, hi=30)
        b.sys_offsets = None
        return b
    if name == "water21k":
        # 7,000 molecules in a 59.6 A box: 17^3 cells at 3.5 A, above the one-work-group
        # binning limit of 4,096 cells, so the list takes the multi-kernel binning
        return synth.water_box(7000, 59.6, seed=21)
    if name == "wrapped1500":
        rng = np.random.default_rng(5)
        pos = rng.uniform(-30.0, 50.0, size=(1500, 3))
        sp = rng.choice(5, size=1500).astype(np.int32)
        return synth.System(pos=pos, species=sp, box=24.0, name="wrapped1500")
    raise KeyError(name)


SPECS = {"small": synth.SMALL, "large": synth.LARGE, "small_mp": synth.SMALL_MP}
SEEDS = {"small": synth.SMALL_SEED, "large": synth.LARGE_SEED, "small_mp": synth.SMALL_MP_SEED}


@functools.lru_cache(maxsize=None)
def weights(which):
    return synth.model_weights(SPECS[which], SEEDS[which])


@functools.lru_cache(maxsize=None)
def oracle_model(which, scale=None):
    s = SPECS[which]
    return OP.make_model(s.kind, s.cutoff, s.n_rbf, s.width, weights(which),
                         energy_scale=s.energy_scale if scale is None else scale)


@functools.lru_cache(maxsize=None)
def oracle_ef(sysname, which):
    sy = system(sysname)
    E, F, Ea = OP.energy_forces(oracle_model(which), sy.pos, sy.species, sy.box, sy.sys_offsets)
    return E, F, Ea


@functools.lru_cache(maxsize=None)
def oracle_pairs(sysname, cutoff):
    sy = system(sysname)
    return ON.pairs(sy.pos, sy.box, cutoff, sy.sys_offsets)


def rel_rmse(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


__all__ = ["say", "system", "weights", "oracle_model", "oracle_ef", "oracle_pairs", "rel_rmse",
           "OI", "OP", "ON", "synth", "SPECS"]
