"""Benchmark of the LJ hot path on one MI355X.

Workload: 32,000,000 particles on a 200^3-cell FCC lattice at number density
0.5 (L = 400), Maxwell-Boltzmann velocities at T = 1 (seed 3), rc = 2.5 with
the Eq. 1 truncation, skin 0.3, dt = 0.005.  A step is one whole velocity-Verlet
step of the hot path: kick, drift, DUTC check, list rebuild when due (cell
binning, counting sort, pair list), pair forces, kick.  The headline is the
FP32-mixed path; the plain FP64 path runs beside it on the same state.

Prints one JSON line.  Timing: HIP events on the library's stream around
exactly K steps after W warm-up steps, with torch.cuda.synchronize() on both
sides.  The force kernel's average launch time comes from the library's own
HIP events (md_set_timing) over the same timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VEC_PEAK_TFLOPS = 157.3   # MI355X vector FP32, published
FP64_VEC_PEAK_TFLOPS = 78.6    # MI355X vector FP64, published
FLOP_PER_PAIR = 25             # dr 3, r^2 5, 1/r^2 1, r^-6 2, scalar 5, f d 3, accumulate i and j 6


def algorithmic_bytes_per_particle_step(rho, r_list):
    """What the force/integrate pass must move per particle and step: FP64 q and v
    read and written (96 B) plus the sorted half pair list of Fig. 1 (4 B per
    unordered pair within r_list: rho * (2 pi / 3) * r_list^3 pairs per particle)."""
    n_half = rho * (2.0 * math.pi / 3.0) * r_list ** 3
    return 96.0 + 4.0 * n_half


def pairs_within_rc_per_particle(rho, rc):
    return rho * (2.0 * math.pi / 3.0) * rc ** 3


def run_gpu(B, torch, w, precision, steps, warmup, tpk=0):
    stream = torch.cuda.Stream()
    p = B.make_params(w.n, w.box, rc=w.rc, skin=w.skin, dt=w.dt, precision=precision, threads_per_key=tpk)
    with torch.cuda.stream(stream):
        ctx = B.Context(p, stream=stream)
        ctx.set_state(w.pos, w.vel)
        t0 = time.time()
        ctx.step(warmup)
        warm_s = time.time() - t0
        st0 = ctx.stats()
        ctx.set_timing(True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = ctx.stats()
        ke, pe = ctx.energy()
        ctx.close()
    return {
        "ms_total": ms,
        "ms_per_step": ms / steps,
        "value": w.n * steps / (ms / 1e3),
        "force_ms_avg": st["force_ms"] / max(st["force_launches"], 1),
        "force_launches": st["force_launches"],
        "rebuild_chain_ms_total": st["rebuild_ms"],
        "rebuilds": st["rebuilds"] - st0["rebuilds"],
        "list_cap": st["list_cap"],
        "max_list_len": st["max_list_len"],
        "threads_per_key": st["threads_per_key"],
        "E_per_particle_end": (ke + pe) / w.n,
        "warmup_s": warm_s,
    }


def cpu_baseline(w, sample_steps):
    """The FP64 oracle, as it stands, on the same 32M state: its initial list
    build plus sample_steps velocity-Verlet steps (DUTC rebuilds included)."""
    import oracle
    t0 = time.time()
    r = oracle.run(w.pos, w.vel, w.box, sample_steps, rc=w.rc, skin=w.skin, dt=w.dt)
    t = time.time() - t0
    return {"value": w.n * sample_steps / t, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP64 CPU oracle on the same %d-particle state: initial cell list + pair list, then %d "
                      "velocity-Verlet steps with DUTC rebuilds (%d builds), %.1f s wall" %
                      (w.n, sample_steps, r.rebuilds, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncell", type=int, default=200, help="FCC cells per side (200 -> 32M particles)")
    ap.add_argument("--tpk", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU form in this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_3450_amd import binding as B
    from paper_1210_3450_amd import inputs

    torch.cuda.set_device(0)
    w = inputs.fcc_workload("fcc%d^3_rho0.5" % args.ncell, args.ncell, seed=3, nsteps=args.steps)
    print("bench: %s, N = %d, L = %g, %d warm-up + %d timed steps" % (w.name, w.n, w.box[0], args.warmup,
                                                                       args.steps), file=sys.stderr, flush=True)
    mixed = run_gpu(B, torch, w, B.MD_PREC_FP32_MIXED, args.steps, args.warmup, args.tpk)
    print("bench: FP32-mixed %.3f ms/step" % mixed["ms_per_step"], file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(B, torch, w, B.MD_PREC_FP64, args.steps, args.warmup, args.tpk)
        print("bench: FP64 %.3f ms/step" % fp64["ms_per_step"], file=sys.stderr, flush=True)

    rho = 0.5
    rl = w.rc + w.skin
    bpp = algorithmic_bytes_per_particle_step(rho, rl)
    pairs = pairs_within_rc_per_particle(rho, w.rc) * w.n
    force_bytes = bpp * w.n
    achieved = force_bytes / (mixed["force_ms_avg"] / 1e3) / 1e9
    gflops = FLOP_PER_PAIR * pairs / (mixed["ms_per_step"] / 1e3) / 1e9

    out = {
        "metric": "particle-steps/s + Gflop/s, 32M LJ, FP32-mixed vs FP64 on 1 MI355X",
        "value": mixed["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair forces / f64 state",
        "data": "synthetic: FCC lattice, Maxwell-Boltzmann velocities (seeded)",
        "config": {"workload": "fcc32M_rho0.5_rc2.5_skin0.3_dt0.005" if args.ncell == 200 else w.name,
                   "n_particles": w.n, "box": w.box[0], "rc": w.rc, "skin": w.skin, "dt": w.dt,
                   "precision": "fp32-mixed", "threads_per_key": mixed["threads_per_key"]},
        "gflops": gflops,
        "pair_flop_convention": "25 flop per unordered pair within rc",
        "mixed": mixed,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_force<FP32_MIXED> (pair forces + kicks + drift)",
                     "bytes_per_particle": bpp, "launch_ms_avg": mixed["force_ms_avg"]},
    }
    if fp64 is not None:
        out["fp64"] = dict(fp64, gflops=FLOP_PER_PAIR * pairs / (fp64["ms_per_step"] / 1e3) / 1e9,
                           force_achieved_gbs=force_bytes / (fp64["force_ms_avg"] / 1e3) / 1e9)
    if not args.no_cpu:
        print("bench: CPU oracle sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
