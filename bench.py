#!/usr/bin/env python3
"""Throughput of the DMTS hot path on one MI355X.

Workload (default): 1,500 H2O (4,500 atoms) in a 35.5 A periodic cube; the one-interaction
fast model (r_c 3.5 A) at a 1 fs inner step and the two-interaction reference model
(r_c 5.2 A) at a 4 fs outer step, FP32 model arithmetic, FP64 integration, NVE.

One timed step = one outer step of Algorithm 1 (4 fs of simulated time): 4 fast-model and
1 reference-model energy+force evaluations, each with its neighbor-list build, plus all
kicks and drifts.  The single-time-step baseline (velocity Verlet, 1 fs, reference model)
is timed on the same GPU over the same simulated time.

Prints one JSON line.  `value` is DMTS ns/day on the one GPU; the line also carries
atom-steps/s (1 step = 1 fs), the Verlet rate and speedup, the force error of both models
against the FP64 oracle, the roofline of the dominant kernel (timed live with HIP events)
and the oracle's own rate on this host's cores.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DMTS ns/day & atom-steps/s vs 1 fs Verlet, same GPU; force RMSE vs FP64"

# Algorithmic work per real pair of each pair kernel, at 2 flops per multiply-add and one
# per add, multiply or transcendental (exp, reciprocal, sine/cosine), counted once per
# pair even where the kernels split the channels over two waves.
# Reference model, interaction t, per channel c (F = 128 channels, K = 32 radial terms):
#   forward:  a = (W_b b)_c + S_c + R_c          2K + 2
#             SiLU(a) = a / (1 + e^-a)           4   (exp, add, reciprocal, multiply)
#             m = f_c SiLU(a)                     1
#             M[y] += m Y_y, 10 components       20
#   backward: a recomputed (2K + 2), sigma = 1 / (1 + e^-a) (3), s = a sigma (1),
#             s' = sigma + s (1 - sigma) (3), m = f_c s (1), dm = sum_y D_y Y_y (20),
#             da = dm f_c s' (2), g' = (W_b b')_c (2K), dm s and da g' accumulated for
#             the radial force (4), G_k += D_{k+1} m for the nine angular terms (18)
#   per pair: b_k and b'_k (forward 4K: shift, square, scale, exp; backward 6K), f_c and
#             f_c' (sine/cosine, forward 4, backward 6), Y (15), the force vector (backward
#             about 30) -> forward 4K + 30, backward 6K + 50.
# Fast model (F = 64, K = 16), per directed pair inside the cutoff:
#   evaluation ("small_forward"): per channel 4K + 17 (a = (W_r b)_c and (W_r b')_c 4K,
#             two table terms 2, sigma 3, SiLU 1, SiLU' 3, m = f_c s 1, the sum into h 1,
#             dm/dr 3, its product with g_i 2), per pair 6K + 34 (b_k and b'_k 6K, f_c and
#             f_c' 6, the float geometry and the unit vector about 28); the readout adds
#             2 x 2 x 64 x 64 flops per atom, not counted here;
#   force gather ("small_backward"): 7 flops per pair (s_ij + s_ji and three products),
#             bound by its 28 bytes per list slot (index, reverse index, record, reverse
#             record's s).
def _ref_fwd(K=32, F=128):
    return F * (2 * K + 27) + 4 * K + 30         # 11,806


def _ref_bwd(K=32, F=128):
    return F * (4 * K + 54) + 6 * K + 50         # 23,538


PAIR_FLOPS = {"pair2_backward": _ref_bwd(), "pair1_backward": _ref_bwd(),
              "pair2_forward": _ref_fwd(), "pair1_forward": _ref_fwd(),
              "small_backward": 7,
              "small_forward": 64 * (4 * 16 + 17) + 6 * 16 + 34}    # 5,314

# The same work split by the pipe that executes it (per pair):
#   radial  the dense contraction W_b b (and W_b b'): matrix cores, in FP32 (the FP32 form,
#           whose exact three-term bfloat16 split issues six bfloat16 products per FP32
#           one) or in bfloat16 (the BF16 form);
#   moment  the ten-component moment contractions (M, dm, G): FP32 matrix cores;
#   valu    the other additions and multiplications, vector units;
#   trans   exponentials, reciprocals, sines and cosines, vector units at a quarter rate.
# Reference model (F = 128, K = 32): forward radial 2KF, moment 20F, valu 5F + 3K + 17,
# trans 2F + K + 2; backward radial 4KF, moment 38F, valu 14F + 5K + 36, trans 2F + K + 2.
# Fast model evaluation (F = 64, K = 16): radial 4KF, valu 15F + 5K + 32, trans 2F + K + 2.
def _pipes(kernel, K, F):
    if kernel.endswith("_forward") and kernel.startswith("pair"):
        return dict(radial=2 * K * F, moment=20 * F, valu=5 * F + 3 * K + 17, trans=2 * F + K + 2)
    if kernel.endswith("_backward") and kernel.startswith("pair"):
        return dict(radial=4 * K * F, moment=38 * F, valu=14 * F + 5 * K + 36,
                    trans=2 * F + K + 2)
    if kernel == "small_forward":
        return dict(radial=4 * K * F, moment=0, valu=15 * F + 5 * K + 32, trans=2 * F + K + 2)
    return dict(radial=0, moment=0, valu=7, trans=0)


# MI355X peaks (published): matrix cores FP32 157.3 TFLOP/s and BF16 2.5 PFLOP/s (dense),
# FP32 vector 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 lanes x 2 flops, transcendentals a
# quarter of the 78.6 T lane-instructions/s, HBM3E 8 TB/s.
# One launch in this many of the dominant kernel is event-timed inside the timed region.
PROF_EVERY = 4

PEAKS = {"mfma_f32": 157.3e12, "mfma_bf16": 2500e12, "valu": 157.3e12, "trans": 19.66e12,
         "hbm": 8e12}


def pipe_roofline(kernel, pairs, seconds, precision, traffic):
    """Per-pipe fractions of one launch of `kernel` and the binding (largest) one.  The
    FP32 matrix and vector pipes of a SIMD do not issue together (measured), so their sum,
    "simd_issue", bounds the launch as well."""
    K, F = (16, 64) if kernel.startswith("small") else (32, 128)
    w = _pipes(kernel, K, F)
    bf16 = precision == "bf16"
    work = {"mfma_f32": pairs * (w["moment"] + (0 if bf16 else w["radial"])),
            "mfma_bf16": pairs * (w["radial"] if bf16 else 0),
            "valu": pairs * w["valu"], "trans": pairs * w["trans"]}
    pipes = {}
    for p, x in work.items():
        if x > 0:
            pipes[p] = {"achieved": x / seconds, "peak": PEAKS[p], "frac": x / seconds / PEAKS[p]}
    if traffic:
        pipes["hbm"] = {"achieved": traffic / seconds, "peak": PEAKS["hbm"],
                        "frac": traffic / seconds / PEAKS["hbm"]}
    issue = sum(v["frac"] for k, v in pipes.items() if k != "hbm")
    bound = max(pipes, key=lambda k: pipes[k]["frac"])
    return bound, pipes, issue


def measured_traffic(workload, precision, kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter summary, or None when
    the summary is for another workload or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2510_06562_amd", "csrc")
    src = "".join(open(os.path.join(csrc, f)).read() for f in ("large.hip", "small.hip", "common.h"))
    if hashlib.sha1(src.encode()).hexdigest()[:16] != rec["hash"]:
        return None
    return rec["bytes"].get(kernel)


def clock_ramp(run, seconds=0.3):
    """Keep the GPU busy with the workload (on scratch copies of the state) for about
    `seconds` before the warm-up steps: the per-launch time of the pair kernels falls by
    ~15% over the first ~50 ms of load while the clocks ramp up."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        run()
        torch.cuda.synchronize()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed outer steps (4 fs each)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="water4500",
                    choices=["water4500", "water192", "solvated100k"])
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the throughput line: time a plain device-to-device copy "
                         "of this many bytes (the reference for hardware byte counters)")
    ap.add_argument("--batch", action="store_true",
                    help="instead of the throughput line: the batched form on 256 open "
                         "molecules (energy+forces of both models) against a per-molecule loop")
    ap.add_argument("--nve-ps", type=float, default=0.0,
                    help="instead of the throughput line: run DMTS and Verlet for this many ps "
                         "of NVE dynamics and report the drift of KE + E_reference")
    ap.add_argument("--gamma", type=float, default=0.0,
                    help="Langevin friction per fs for both timed runs (0: NVE; the paper's "
                         "production value is 0.001)")
    ap.add_argument("--temperature", type=float, default=300.0)
    ap.add_argument("--fast-model", default="one", choices=["one", "mp"],
                    help="fast model: one interaction (rc 3.5 A, F 64; default) or the "
                         "message-passing variant (two interactions as the reference model, "
                         "rc 3.5 A), which runs on the shared list filtered to 3.5 A")
    ap.add_argument("--hmr", action="store_true",
                    help="hydrogen mass repartitioning (3.024 amu hydrogens, mass taken from "
                         "the nearest heavy atom) for every dynamics run")
    ap.add_argument("--distill", action="store_true",
                    help="fit the fast model's readout vector to the reference energies and "
                         "forces on frames of a reference-model run before timing, and "
                         "report the slow force's autocorrelation before and after")
    ap.add_argument("--n-inner", type=int, default=4)
    ap.add_argument("--dt-inner", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verlet", action="store_true")
    ap.add_argument("--distill-frames", type=int, default=16,
                    help="frames of the reference run the readout is fitted on (50 fs apart)")
    ap.add_argument("--no-nve", action="store_true",
                    help="skip the 10 ps NVE drift run of the throughput line")
    ap.add_argument("--skin", type=float, default=None,
                    help="skin of the reference lists in A (default: the library's)")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the 100,001-atom BF16 DMTS and 256-molecule BF16 batch lines "
                         "that the default water4500 run adds (child processes)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shapes instead of tuning them for the workload")
    ap.add_argument("--shapes", default=None,
                    help='JSON {"fast": {...}, "reference": {...}} of tile shapes to use instead '
                         "of tuning (keys as in the line's tile_shapes), e.g. to profile the "
                         "shapes an unprofiled run chose: a profiler's per-launch overhead can "
                         "change the tuner's ranking")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="MLP contraction operands (bf16: bfloat16 operands, FP32 accumulate)")
    return ap.parse_args()


def host_cpu():
    """(logical CPUs this process may use, the CPU model name of the host)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:  # pragma: no cover
        pass
    return n, model


def cpu_oracle(sy, ws, wl, n_inner, dt_inner, spec_s, spec_l, synth):
    """Time the FP64 oracle on this host (the bounded sample): the median of three
    fast-model and three reference-model evaluations of the workload with every BLAS thread,
    extrapolated to DMTS ns/day; the same pair of evaluations of the 192-atom box on one
    thread, scaled per atom to the workload; and the 192-atom box's 20-step velocity-Verlet
    run (0.5 fs, fast model)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import integrators as OI
    from oracle import potentials as OP

    cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    nproc, model = host_cpu()
    ms = OP.make_model(spec_s.kind, spec_s.cutoff, spec_s.n_rbf, spec_s.width, ws,
                       energy_scale=spec_s.energy_scale)
    ml = OP.make_model(spec_l.kind, spec_l.cutoff, spec_l.n_rbf, spec_l.width, wl,
                       energy_scale=spec_l.energy_scale)

    def timed(model_, s):
        t0 = time.perf_counter()
        r = OP.energy_forces(model_, s.pos, s.species, s.box)
        return time.perf_counter() - t0, r

    runs_s = [timed(ms, sy) for _ in range(3)]
    runs_l = [timed(ml, sy) for _ in range(3)]
    t_s = float(np.median([t for t, _ in runs_s]))
    t_l = float(np.median([t for t, _ in runs_l]))
    Es, Fs, _ = runs_s[0][1]
    El, Fl, _ = runs_l[0][1]
    outer_fs = n_inner * dt_inner
    small_box = synth.water_192()
    with threadpool_limits(limits=1):
        t1_s = timed(ms, small_box)[0]
        t1_l = timed(ml, small_box)[0]
    per_atom = (n_inner * t1_s + t1_l) / small_box.n_atoms
    # the 192-atom box's reference run: 1 evaluation + 20 velocity-Verlet steps at 0.5 fs
    st = OI.MTSState(x=small_box.pos.copy(), v=synth.maxwell_boltzmann(small_box.species, 300.0, 200),
                     m=small_box.masses())
    f = lambda x: (lambda r: (r[0][0], r[1]))(OP.energy_forces(ms, x, small_box.species,  # noqa: E731
                                                                  small_box.box))
    t0 = time.perf_counter()
    OI.sts_step(st, 0.0, f)
    for _ in range(20):
        OI.sts_step(st, 0.5, f)
    t_c0 = time.perf_counter() - t0
    return dict(t_small=t_s, t_large=t_l, cores=cores, nproc=nproc, cpu_model=model,
                ns_per_day=0.0864 * outer_fs / (n_inner * t_s + t_l),
                ns_per_day_1_thread=0.0864 * outer_fs / (per_atom * sy.n_atoms),
                t1_small_192=t1_s, t1_large_192=t1_l, c0_run_s=t_c0,
                Es=Es, Fs=Fs, El=El, Fl=Fl)


def drift_fit(t_ps, H, n_atoms, span_ps):
    """Least-squares line through H(t): (drift over span_ps per atom, its standard error,
    the largest |H - H(0)| per atom).  The residuals of H are serially correlated (its
    fluctuations last longer than the sampling interval), so the ordinary least-squares
    error is widened by the AR(1) factor sqrt((1 + rho) / (1 - rho)), rho the lag-one
    autocorrelation of the residuals (kept >= 0)."""
    A = np.vstack([t_ps, np.ones_like(t_ps)]).T
    coef = np.linalg.lstsq(A, H, rcond=None)[0]
    resid = H - A @ coef
    se = np.sqrt(resid @ resid / max(len(H) - 2, 1) / np.sum((t_ps - t_ps.mean()) ** 2))
    rho = float(resid[1:] @ resid[:-1] / max(resid @ resid, 1e-300)) if len(H) > 2 else 0.0
    rho = min(max(rho, 0.0), 0.99)
    se *= np.sqrt((1.0 + rho) / (1.0 - rho))
    return (float(coef[0] * span_ps / n_atoms), float(se * span_ps / n_atoms),
            float(np.max(np.abs(H - H[0])) / n_atoms))


def nve_10ps(api, synth, sy, sp, v0, small, large, dt_outer, n_inner, masses=None):
    """10 ps of NVE DMTS from the workload's start, H = KE + E_reference every ~20 fs: the
    drift criterion's figures (drift over 10 ps per atom, the fit's standard error, the
    largest deviation) and the fallback count."""
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt_outer, n_inner, 64, 128)
    if masses is not None:
        st.set_atom_masses(masses)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    n_steps = int(round(10000.0 / dt_outer))
    chunk = max(1, int(round(20.0 / dt_outer)))
    t, H = [0.0], [st.step(x, v, small, large, 0)[3].item()]
    done = 0
    t0 = time.perf_counter()
    while done < n_steps:
        k = min(chunk, n_steps - done)
        H.append(st.step(x, v, small, large, k)[3].item())
        done += k
        t.append(done * dt_outer / 1000.0)
    drift, se, dev = drift_fit(np.array(t), np.array(H), sy.n_atoms, 10.0)
    return {"drift_eV_per_atom": drift, "drift_se_eV_per_atom": se, "max_dev_eV_per_atom": dev,
            "samples": len(H), "outer_steps": n_steps, "fallbacks": st.fallbacks,
            "wall_s": round(time.perf_counter() - t0, 2)}


def nve_drift(args, api, synth, sy, sp, v0, small, large):
    """NVE runs of DMTS (dt_inner / n_inner) and of 1 fs Verlet (reference model): the
    conserved energy H = KE + E_reference sampled every outer step, its least-squares slope
    and the drift over the run per atom."""
    import torch

    out = {"mode": "nve-drift", "workload": args.workload, "n_atoms": sy.n_atoms,
           "precision": args.precision, "ps": args.nve_ps, "hmr": args.hmr,
           "fast_model": args.fast_model, "distilled": args.distill}
    for name, small_m, dt, n_in in (("dmts", small, args.dt_inner * args.n_inner, args.n_inner),
                                    ("verlet", None, args.dt_inner, 1)):
        st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt, n_in, 64, 128)
        if args.hmr:
            st.set_atom_masses(sy.hmr_masses())
        x, v = api.to_soa(sy.pos), api.to_soa(v0)
        n_steps = int(round(args.nve_ps * 1000.0 / dt))
        chunk = max(1, int(round(20.0 / dt)))   # sample every ~20 fs
        t, H = [0.0], [st.step(x, v, small_m, large, 0)[3].item()]
        done = 0
        t0 = time.perf_counter()
        while done < n_steps:
            k = min(chunk, n_steps - done)
            H.append(st.step(x, v, small_m, large, k)[3].item())
            done += k
            t.append(done * dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t, H = np.array(t) / 1000.0, np.array(H)      # ps, eV
        slope = np.polyfit(t, H, 1)[0]
        out[name] = {"slope_eV_per_atom_per_ps": slope / sy.n_atoms,
                     "drift_eV_per_atom": slope * args.nve_ps / sy.n_atoms,
                     "max_dev_eV_per_atom": float(np.max(np.abs(H - H[0]))) / sy.n_atoms,
                     "kT_eV": 8.617333262e-5 * 300.0, "steps": n_steps, "dt_fs": dt,
                     "wall_s": wall, "fallbacks": st.fallbacks}
        print(f"{name}: {n_steps} steps in {wall:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def batch_throughput(args, api, synth, small, large):
    """256 open molecules (20-120 atoms): energy and forces of both models, batched in one
    launch per kernel with an autotuned persistent grid, against a loop that evaluates one
    molecule at a time.  Reports molecules/s and atom-evaluations/s of both."""
    import torch

    sy = synth.molecule_batch(256, 3)
    pos = api.to_soa(sy.pos)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    offs = torch.as_tensor(sy.sys_offsets, dtype=torch.int32, device="cuda")
    pots = [api.Potential(m, sy.n_atoms, 0.0, 160, offs, check=False) for m in (small, large)]
    tuned = [api.autotune(p, pos, sp, reps=3) for p in pots]
    reps = max(args.steps, 3)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return max(ev0.elapsed_time(ev1), (time.perf_counter() - t0) * 1e3) / reps

    def batched():
        for p in pots:
            p(pos, sp)

    ones = [api.Potential(m, 128, 0.0, 160, check=False) for m in (small, large)]
    mols = [(api.to_soa(sy.pos[a:b]), sp[a:b].contiguous())
            for a, b in zip(sy.sys_offsets[:-1], sy.sys_offsets[1:])]

    def loop():
        for pm, sm in mols:
            for p in ones:
                p(pm, sm)

    t_b = timed(batched)
    t_l = timed(loop)
    out = {"mode": "batch", "molecules": 256, "n_atoms": sy.n_atoms,
           "precision": args.precision, "tuned_shapes": {"fast": tuned[0][0],
                                                        "reference": tuned[1][0]},
           "batched_ms": round(t_b, 4), "per_molecule_loop_ms": round(t_l, 4),
           "batched_molecules_per_s": round(256 / (t_b * 1e-3), 1),
           "loop_molecules_per_s": round(256 / (t_l * 1e-3), 1),
           "batched_atom_evals_per_s": round(sy.n_atoms / (t_b * 1e-3), 1),
           "speedup": round(t_l / t_b, 2)}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-GPU: one process drives one device.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_06562_amd import api, synth

    torch.cuda.set_device(0)
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"mode": "copy", "bytes": args.copy_bytes,
                          "GBps_read_plus_write": 2 * args.copy_bytes / dt / 1e9}), flush=True)
        return
    sy = {"water4500": synth.water_4500, "water192": synth.water_192,
          "solvated100k": synth.solvated_chain}[args.workload]()
    spec_s, seed_s = ((synth.SMALL, synth.SMALL_SEED) if args.fast_model == "one" else
                      (synth.SMALL_MP, synth.SMALL_MP_SEED))
    ws = synth.model_weights(spec_s, seed_s)
    wl = synth.model_weights(synth.LARGE, synth.LARGE_SEED)
    prec = api.PREC_BF16 if args.precision == "bf16" else api.PREC_FP32
    large = api.Model.from_spec(synth.LARGE, wl, precision=prec)
    sp = torch.as_tensor(sy.species, dtype=torch.int32, device="cuda")
    v0 = synth.maxwell_boltzmann(sy.species, 300.0, 201,
                                 masses=sy.hmr_masses() if args.hmr else None)
    distilled = None
    atom_masses = sy.hmr_masses() if args.hmr else None
    if args.distill:
        from paper_2510_06562_amd import distill
        # frames 50 fs apart over 800 fs of reference dynamics (with the run's masses)
        snaps = distill.reference_snapshots(large, sp, sy.box, synth.MASSES, sy.pos, v0,
                                            args.distill_frames, 50, atom_masses=atom_masses)
        acf = lambda w_: distill.slow_force_autocorrelation(  # noqa: E731
            large, api.Model.from_spec(spec_s, w_, precision=prec), sp, sy.box, synth.MASSES,
            sy.pos, v0, 400, 1.0, atom_masses)
        before = acf(ws)
        ws, distilled = distill.fit_readout(spec_s, ws, large, sp, sy.box, snaps,
                                            precision=prec)
        distilled["slow_force_before"] = before
        distilled["slow_force_after"] = acf(ws)
        print(f"distilled readout: rms |F_L - F_S| {distilled['rms_before']:.5f} -> "
              f"{distilled['rms_after']:.5f} eV/A; tau_int {before['tau_int_fs']:.2f} -> "
              f"{distilled['slow_force_after']['tau_int_fs']:.2f} fs", file=sys.stderr,
              flush=True)
    small = api.Model.from_spec(spec_s, ws, precision=prec)
    n_inner, dt_in = args.n_inner, args.dt_inner
    dt_out = n_inner * dt_in
    stream = torch.cuda.current_stream()
    if args.nve_ps > 0:
        return nve_drift(args, api, synth, sy, sp, v0, small, large)
    if args.batch:
        return batch_throughput(args, api, synth, small, large)

    # ---------------------------------------------------------------- GPU forces for the error
    pot_s = api.Potential(small, sy.n_atoms, sy.box, 64)
    pot_l = api.Potential(large, sy.n_atoms, sy.box, 128)
    x0 = api.to_soa(sy.pos)
    Es_gpu, Fs_gpu = pot_s(x0, sp)
    El_gpu, Fl_gpu = pot_l(x0, sp)
    offs, nbr, _ = pot_l.nlist.download(sy.n_atoms)
    pairs_large = int(np.sum(nbr >= 0))
    offs_s, nbr_s, _ = pot_s.nlist.download(sy.n_atoms)
    pairs_small = int(np.sum(nbr_s >= 0))

    # ---------------------------------------------------------------- tile shapes
    # each model's shape for this system size, tuned on the list it runs on in the RESPA
    # loop (the reference model's cutoff, shared by the fast model)
    shapes = {}
    if args.shapes:
        given = json.loads(args.shapes)
        for name, mdl in (("fast", small), ("reference", large)):
            if name in given:
                sh = {k: int(v) for k, v in given[name].items()
                      if k in ("receivers_per_group", "atom_tiles", "keep_derivatives",
                               "work_groups")}
                mdl.set_shape(sy.n_atoms, **sh)
                shapes[name] = dict(mdl.shape(sy.n_atoms), given=True)
    elif not args.no_autotune:
        list_cut = max(synth.LARGE.cutoff, spec_s.cutoff + 1.0)
        for name, mdl in (("fast", small), ("reference", large)):
            p = api.Potential(mdl, sy.n_atoms, sy.box, 128)
            sh, t = api.autotune(p, x0, sp, reps=3, cutoff=list_cut)
            shapes[name] = dict(sh, ms=round(t, 4))

    # ---------------------------------------------------------------- DMTS timed region
    st = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt_out, n_inner, 64, 128)
    if args.skin is not None:
        st.set_skin(args.skin)
    if args.hmr:
        st.set_atom_masses(sy.hmr_masses())
    if args.gamma > 0.0:
        st.set_thermostat(args.gamma, args.temperature, 2025)
    x, v = api.to_soa(sy.pos), api.to_soa(v0)
    clock_ramp(lambda: st.step(x.clone(), v.clone(), small, large, 4))
    st.reset()
    st.step(x, v, small, large, max(args.warmup, 1))
    torch.cuda.synchronize()
    # kernel census (all classes timed); the roofline is taken on the pair kernel with the
    # longest launches (the reference model's reverse pass), whose event-timed duration
    # carries the least launch overhead
    api.prof_reset()
    api.prof_enable(None)
    st.step(x, v, small, large, 2)
    census = api.prof_read()
    api.prof_enable(())
    api.prof_reset()
    timed = {k: census[k] for k in PAIR_FLOPS if census[k][1] > 0}
    dom = max(timed, key=lambda k: timed[k][0] / timed[k][1]) if timed else None
    torch.cuda.synchronize()
    H_start = st.energies[3].item()
    # the dominant kernel is timed live in the timed region on one launch in PROF_EVERY:
    # each timed dispatch records its two events in its own packet, which idles the
    # queue for ~5 us on either side of it
    api.prof_enable([dom] if dom else ())
    api.prof_sample(PROF_EVERY)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    builds0 = st.list_builds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    st.step(x, v, small, large, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    list_builds = st.list_builds - builds0
    api.prof_enable(())
    prof = api.prof_read()
    api.prof_sample(1)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_step = max(gpu_ms, wall * 1e3) / args.steps
    H_end = st.energies[3].item()
    sim_fs = dt_out
    ns_day = 0.0864 * sim_fs / (ms_step * 1e-3)
    atom_steps = sy.n_atoms * (sim_fs / dt_in) / (ms_step * 1e-3)

    # ---------------------------------------------------------------- Verlet, same GPU
    vv = None
    if not args.no_verlet:
        st_v = api.DMTS(sy.n_atoms, sy.box, sp, synth.MASSES, dt_in, 1, 64, 128)
        st_v.set_skin(st.skin)
        if args.hmr:
            st_v.set_atom_masses(sy.hmr_masses())
        if args.gamma > 0.0:
            st_v.set_thermostat(args.gamma, args.temperature, 2026)
        xv, vvel = api.to_soa(sy.pos), api.to_soa(v0)
        st_v.step(xv, vvel, None, large, max(args.warmup, 1))
        torch.cuda.synchronize()
        n_vv = args.steps * n_inner
        vb0 = st_v.list_builds
        t0 = time.perf_counter()
        ev0.record(stream)
        st_v.step(xv, vvel, None, large, n_vv)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall_v = time.perf_counter() - t0
        ms_vv = max(ev0.elapsed_time(ev1), wall_v * 1e3) / n_vv
        vv = dict(ns_per_day=0.0864 * dt_in / (ms_vv * 1e-3), ms_per_step=ms_vv,
                  list_builds=st_v.list_builds - vb0, evaluations=n_vv)

    # ---------------------------------------------------------------- 10 ps NVE drift
    nve = None
    if args.gamma <= 0.0 and not args.no_nve:
        nve = nve_10ps(api, synth, sy, sp, v0, small, large, dt_out, n_inner,
                       sy.hmr_masses() if args.hmr else None)

    # ---------------------------------------------------------------- dominant kernel roofline
    roofline = None
    # (with the message-passing fast model both models launch the pair kernels, whose
    # timing classes then mix two pair counts: no roofline line)
    if dom and prof[dom][1] > 0 and args.fast_model == "one":
        tot_ms, launches = prof[dom]
        avg_s = tot_ms / launches * 1e-3
        pairs = pairs_small if dom.startswith("small") else pairs_large
        traffic = measured_traffic(args.workload, args.precision, dom)
        bound, pipes, issue = pipe_roofline(dom, pairs, avg_s, args.precision, traffic)
        b = pipes[bound]
        tera = 1e12
        roofline = {"bound": "hbm" if bound == "hbm" else ("mfma" if bound.startswith("mfma")
                                                           else "alu"),
                    "pipe": bound, "kernel": dom,
                    "achieved": round(b["achieved"] / tera, 3), "peak": round(b["peak"] / tera, 2),
                    "unit": "TB/s" if bound == "hbm" else "TFLOP/s",
                    "frac": round(b["frac"], 4), "traffic": traffic,
                    "pipes": {k: {"achieved_T": round(v["achieved"] / tera, 3),
                                  "peak_T": round(v["peak"] / tera, 2), "frac": round(v["frac"], 4)}
                              for k, v in pipes.items()},
                    "simd_issue_frac": round(issue, 4),
                    "avg_launch_us": round(avg_s * 1e6, 2), "timed_launches": launches,
                    "timed_every": PROF_EVERY, "pairs_per_launch": pairs,
                    "flops_per_pair": PAIR_FLOPS[dom]}

    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        c = cpu_oracle(sy, ws, wl, n_inner, dt_in, spec_s, synth.LARGE, synth)
        cpu = {"value": round(c["ns_per_day"], 6), "unit": "ns/day", "cores": c["cores"],
               "kind": "oracle", "nproc": c["nproc"], "cpu_model": c["cpu_model"],
               "value_1_thread": round(c["ns_per_day_1_thread"], 6),
               "c0_20_step_run_s": round(c["c0_run_s"], 3),
               "sample": (f"median of three fast-model ({c['t_small']:.2f} s) and three "
                          f"reference-model ({c['t_large']:.2f} s) FP64 energy+force "
                          f"evaluations of the {sy.n_atoms}-atom box on {c['cores']} BLAS "
                          f"threads, extrapolated to one {dt_out:g} fs outer step ({n_inner} "
                          f"fast + 1 reference evaluation); value_1_thread: one thread, the "
                          f"192-atom box ({c['t1_small_192']:.3f} s + {c['t1_large_192']:.3f} s) "
                          f"scaled per atom; c0_20_step_run_s: the 192-atom box, 1 evaluation "
                          f"+ 20 velocity-Verlet steps of 0.5 fs with the fast model")}
        Fs_np, Fl_np = api.from_soa(Fs_gpu), api.from_soa(Fl_gpu)
        errors = {
            "force_rel_rmse_small": float(np.linalg.norm(Fs_np - c["Fs"]) / np.linalg.norm(c["Fs"])),
            "force_rel_rmse_large": float(np.linalg.norm(Fl_np - c["Fl"]) / np.linalg.norm(c["Fl"])),
            "energy_err_per_atom_small": abs(Es_gpu.item() - c["Es"][0]) / sy.n_atoms,
            "energy_err_per_atom_large": abs(El_gpu.item() - c["El"][0]) / sy.n_atoms,
        }

    kernels = {k: {"ms_per_outer_step": round(t / 2, 4), "launches": n, "us_avg": round(1e3 * t / n, 2)}
               for k, (t, n) in census.items() if n > 0}
    out = {
        "metric": METRIC,
        "value": round(ns_day, 4),
        "unit": "ns/day",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": sy.n_atoms, "box_A": sy.box,
                   "dt_inner_fs": dt_in, "dt_outer_fs": dt_out,
                   "fast_model": ("1 interaction, rc 3.5 A, K 16, F 64" if args.fast_model == "one"
                                  else "2 interactions, rc 3.5 A, K 32, F 128, l<=2"),
                   "reference_model": "2 interactions, rc 5.2 A, K 32, F 128, l<=2",
                   "integration": "f64",
                   "masses": "repartitioned (HMR)" if args.hmr else "species",
                   "ensemble": ("NVE" if args.gamma <= 0.0 else
                                f"Langevin gamma {args.gamma} /fs, {args.temperature} K"),
                   "mlp_operands": args.precision},
        "atom_steps_per_s": round(atom_steps, 1),
        "verlet_ns_per_day": round(vv["ns_per_day"], 4) if vv else None,
        "verlet_ms_per_step": round(vv["ms_per_step"], 5) if vv else None,
        "list_rebuilds": {"skin_A": st.skin,
                          "dmts": {"rebuilds": list_builds, "reference_evaluations": args.steps,
                                   "simulated_fs": args.steps * dt_out},
                          "verlet": ({"rebuilds": vv["list_builds"],
                                      "reference_evaluations": vv["evaluations"],
                                      "simulated_fs": vv["evaluations"] * dt_in} if vv else None)},
        "speedup_vs_verlet": round(ns_day / vv["ns_per_day"], 3) if vv else None,
        "errors_vs_fp64": errors,
        "energy_drift_per_atom": (H_end - H_start) / sy.n_atoms if args.gamma <= 0.0 else None,
        "nve_10ps": nve,
        "pairs": {"fast": pairs_small, "reference": pairs_large},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "distilled_readout": distilled,
        "tile_shapes": shapes,
        "kernels": kernels,
    }
    if (args.workload == "water4500" and not args.no_other_configs and args.fast_model == "one"
            and not (args.hmr or args.distill or args.gamma > 0.0)):
        out["other_configs"] = other_configs(args.precision)
    print(json.dumps(out), flush=True)


def other_configs(precision):
    """The two other workloads of the benchmark set, each run by a child process of this
    script: DMTS 1 fs / 6 fs against 1 fs Verlet on the 100,001-atom solvated chain, and
    one batched evaluation of 256 molecules against a per-molecule loop, both with BF16
    MLP operands (the forms those workloads are specified in).  Returns a summary of each
    child's JSON line (or the error it ended with)."""
    import subprocess

    def child(extra, keys):
        cmd = [sys.executable, os.path.abspath(__file__), "--no-other-configs", *extra]
        try:
            r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        except subprocess.TimeoutExpired:
            return {"error": "timed out", "command": " ".join(extra)}
        lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
        if r.returncode != 0 or not lines:
            return {"error": f"exit {r.returncode}", "command": " ".join(extra),
                    "stderr_tail": r.stderr[-400:]}
        d = json.loads(lines[-1])
        o = {k: d.get(k) for k in keys}
        o["command"] = "bench.py " + " ".join(extra)
        return o

    c4 = child(["--workload", "solvated100k", "--precision", "bf16", "--n-inner", "6",
                "--steps", "5", "--warmup", "2", "--no-cpu-baseline", "--no-nve"],
               ("metric", "value", "unit", "ms_per_step", "dtype", "config", "atom_steps_per_s",
                "verlet_ns_per_day", "verlet_ms_per_step", "speedup_vs_verlet", "list_rebuilds",
                "roofline"))
    c3 = child(["--batch", "--precision", "bf16"],
               ("molecules", "n_atoms", "precision", "tuned_shapes", "batched_ms",
                "per_molecule_loop_ms", "batched_molecules_per_s", "loop_molecules_per_s",
                "batched_atom_evals_per_s", "speedup"))
    return {"solvated100k_bf16_dmts": c4, "batch256_bf16": c3}


if __name__ == "__main__":
    main()
