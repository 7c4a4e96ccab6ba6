"""The reference evaluations' lists through the skin list: rows kept at cutoff + skin and
rebuilt only when some atom has moved half the skin, filtered to the cutoff at every
evaluation.  The filtered rows are those of a fresh build, so a run with a skin equals the
run that builds afresh at every evaluation (skin 0) bit for bit, while rebuilding the rows
only now and then.  The oracle comparisons of the other dynamics tests run with the default
skin as well."""

import numpy as np
import pytest
import torch

from _gpu_common import say, system, weights, SPECS
from paper_2510_06562_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def models():
    return {k: api.Model.from_spec(SPECS[k], weights(k)) for k in ("small", "large")}


def _run(sy, small, large, dt, n_inner, n_outer, skin):
    """x, v after n_outer outer steps, and the row rebuilds."""
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_inner, 48, 128)
    st.set_skin(skin)
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    st.step(x, v, small, large, n_outer)
    torch.cuda.synchronize()
    return x, v, st.list_builds


@pytest.mark.parametrize("name", ["water192", "water4500"])
def test_dmts_with_skin_equals_fresh_builds(models, name):
    """40 fs of DMTS (1 fs / 4 fs): identical bits with the 1 A skin and with fresh builds;
    the rows are rebuilt at most at eight of the eleven reference evaluations (water192 has fewer
    than three cells per edge at 6.2 A, so its rows come from the all-pairs search)."""
    say(f"skin vs fresh builds, DMTS {name}")
    sy = system(name)
    x0, v0, b0 = _run(sy, models["small"], models["large"], 4.0, 4, 10, 0.0)
    x1, v1, b1 = _run(sy, models["small"], models["large"], 4.0, 4, 10, 1.0)
    say(f"  row rebuilds over 11 reference evaluations: {b1}")
    assert b0 == 0
    assert torch.equal(x0, x1) and torch.equal(v0, v1)
    assert 1 <= b1 <= 8


def test_verlet_with_skin_equals_fresh_builds(models):
    """The single-time-step baseline (reference model, 1 fs): 30 steps, the same bits, and
    rows rebuilt well below once per step."""
    say("skin vs fresh builds, velocity Verlet water4500")
    sy = system("water4500")
    x0, v0, _ = _run(sy, None, models["large"], 1.0, 1, 30, 0.0)
    x1, v1, b1 = _run(sy, None, models["large"], 1.0, 1, 30, 1.0)
    say(f"  row rebuilds over 31 evaluations: {b1}")
    assert torch.equal(x0, x1) and torch.equal(v0, v1)
    assert 1 <= b1 <= 10


def test_moved_atoms_force_a_rebuild(models):
    """A rigid shift of every atom by 0.6 A between two calls (more than half the skin for
    every atom whose own motion since the last rebuild has a positive x component) makes
    the next evaluation rebuild the rows; the run still equals the fresh-build one bit for
    bit."""
    say("skin: shifted atoms between calls, water4500")
    sy = system("water4500")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
    out = {}
    for skin in (0.0, 1.0):
        st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, 4.0, 4, 48, 128)
        st.set_skin(skin)
        x, v = api.to_soa(sy.pos), api.to_soa(v0)
        st.step(x, v, models["small"], models["large"], 2)
        before = st.list_builds
        x[0] += 0.6
        st.reset()
        st.step(x, v, models["small"], models["large"], 1)
        out[skin] = (x, v, before, st.list_builds)
    x0, v0_, _, _ = out[0.0]
    x1, v1, before, after = out[1.0]
    assert torch.equal(x0, x1) and torch.equal(v0_, v1)
    assert after >= before + 1


def test_multi_kernel_binning_with_skin(models):
    """Above 32,768 atoms the skin rows take the multi-work-group binning and the filtered
    list the separate offset scan: 11,000 waters (33,000 atoms), 3 outer steps."""
    say("skin vs fresh builds, water33k")
    sy = synth.water_box(11000, 69.1, seed=33)
    x0, v0, _ = _run(sy, models["small"], models["large"], 4.0, 4, 3, 0.0)
    x1, v1, b1 = _run(sy, models["small"], models["large"], 4.0, 4, 3, 1.0)
    assert torch.equal(x0, x1) and torch.equal(v0, v1)
    assert 1 <= b1 <= 4


def test_skin_argument_checks(models):
    sy = system("water192")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, 4.0, 4, 48, 128)
    for bad in (-0.5, float("nan"), float("inf")):
        with pytest.raises(api.DmtsError):
            st.set_skin(bad)
    st.set_skin(0.0)
    st.set_skin(2.0)


def test_skin_with_monitor_and_fallbacks_equals_fresh_builds(models):
    """The skin list under the other paths that roll a call back: a force-difference
    threshold low enough that steps breach (rolled back and redone as single-time-step
    steps), and one fast atom that outruns the shared list's margin (the call is redone
    with exact lists).  Both redo paths see the same lists with the skin as without."""
    say("skin with monitor and fallbacks, water4500")
    sy = system("water4500")
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    for case, thr, fast in (("monitor", 0.02, False), ("fallback", 0.0, True)):
        v0 = synth.maxwell_boltzmann(sy.species, 300.0, 200)
        if fast:
            v0[10] = [0.35, 0.0, 0.0]   # ~1.4 A per 4 fs outer step: past the 0.85 A margin
        out = {}
        for skin in (0.0, 1.5):
            st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, 4.0, 4, 48, 128)
            st.set_skin(skin)
            st.set_fdiff_threshold(thr)
            x, v = api.to_soa(sy.pos), api.to_soa(v0)
            st.step(x, v, models["small"], models["large"], 3)
            torch.cuda.synchronize()
            out[skin] = (x, v, st.fdiff[0], st.fallbacks, st.list_builds)
        x0, v0_, redo0, fb0, _ = out[0.0]
        x1, v1, redo1, fb1, b1 = out[1.5]
        say(f"  {case}: single-time-step redos {redo1}, exact-list fallbacks {fb1}, "
            f"row rebuilds {b1}")
        assert redo0 == redo1 and fb0 == fb1
        assert (redo1 >= 1) if case == "monitor" else (fb1 >= 1)
        assert torch.equal(x0, x1) and torch.equal(v0_, v1)


def test_dense_box_skin_rows_past_the_list_row_limit(models):
    """A jittered lattice at 0.25 atoms/A^3 (2.5 times water, 6,859 atoms): rows hold ~150
    entries at 5.2 A but ~320 at 6.7 A, past a list row's 256 entries.  The skin rows hold
    up to 512, so the run neither overflows nor differs from the fresh-build one."""
    say("skin rows past 256 entries, dense lattice")
    n_side, box = 19, 30.0
    rng = np.random.default_rng(41)
    g = (np.arange(n_side) + 0.5) * (box / n_side)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pos = pos + rng.normal(0.0, 0.1, pos.shape)
    species = rng.choice(5, size=len(pos)).astype(np.int32)
    sp = torch.as_tensor(species, dtype=torch.int32, device="cuda")
    v0 = synth.maxwell_boltzmann(species, 300.0, 7)
    out = {}
    for skin in (0.0, 1.5):
        st = api.DMTS(len(pos), box, sp, synth.MASSES, 4.0, 4, 64, 200)
        st.set_skin(skin)
        x, v = api.to_soa(pos), api.to_soa(v0)
        st.step(x, v, models["small"], models["large"], 2)
        torch.cuda.synchronize()
        out[skin] = (x, v, st.list_builds)
    assert out[1.5][2] >= 1
    assert torch.equal(out[0.0][0], out[1.5][0]) and torch.equal(out[0.0][1], out[1.5][1])
