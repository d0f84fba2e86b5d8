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

Beside the headline the default run adds: the same 32M box with the
displacement rebuild rule, compact figures of the 4000-particle FP64 box
(100 steps), the 1M box in both precisions (100 steps) and the 256-box
ensemble (autotuned, captured graphs) with a one-box-at-a-time baseline on a
subset, and the FP64 CPU oracle on a bounded sample of the 32M run.
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


REBUILD_BYTES_PER_PARTICLE = 260.0  # binning 32, permute 104, list build 124 (per particle per rebuild)
MIXED_NOTE = ("pair forces in FP32 on exact fixed-point cell-relative separations; positions, velocities, "
              "integration and energy totals in FP64")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_t_fcc32m_hbm_traffic.txt")
FLOPS_FILE = os.path.join(ROOT, "profiles", "k_force_t_fcc32m_valu_flops.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1210_3450_amd", "csrc", f) for f in ("md_kernels.hip", "md_internal.h")]


def kernel_source_hash():
    """SHA-256 of the kernel sources with comments and blank lines removed, so that a
    change of wording in a comment does not disown the counters of an unchanged kernel."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = re.sub(r"//.*", "", line).rstrip()
            if line.strip():
                h.update(line.encode() + b"\n")
    return h.hexdigest()


def summary_value(path, key):
    """A "key: value" figure of a committed counter summary, or None when the
    kernel sources changed since the counters were taken (or it is absent)."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) == 2 and parts[0].endswith(":"):
                    kv[parts[0][:-1]] = parts[1]
        if kv.get("kernel_sources_sha256") != kernel_source_hash():
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per force launch (TCC-to-memory read and write requests by size)."""
    return summary_value(TRAFFIC_FILE, "hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_gpu(B, torch, w, precision, steps, warmup, tpk=0, flags=0, rebuild=0):
    stream = torch.cuda.Stream()
    p = B.make_params(w.n, w.box, rc=w.rc, skin=w.skin, dt=w.dt, precision=precision, threads_per_key=tpk,
                      flags=flags, rebuild=rebuild)
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
        "row_tiles": st["row_tiles"],
        "E_per_particle_end": (ke + pe) / w.n,
        "warmup_s": warm_s,
    }


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of a plain
    torch copy_ of nbytes, the best of reps, as the practical HBM ceiling."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best / 1e3) / 1e9


def cpu_baseline(w, sample_steps):
    """The FP64 oracle, as it stands, on the same 32M state: its initial list
    build plus sample_steps velocity-Verlet steps (DUTC rebuilds included), so
    that the sample holds list builds in about the share the GPU run has."""
    import oracle
    t0 = time.time()
    r = oracle.run(w.pos, w.vel, w.box, sample_steps, rc=w.rc, skin=w.skin, dt=w.dt)
    t = time.time() - t0
    return {"value": w.n * sample_steps / t, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "steps": int(r.steps), "list_builds": int(r.rebuilds),
            "dutc_rebuilds": int(r.rebuilds) - 1, "wall_s": t,
            "cpu_model": cpu_model(),
            "sample": "FP64 CPU oracle on the same %d-particle state: initial cell list + pair list, then %d "
                      "velocity-Verlet steps with %d DUTC rebuilds (%d list builds in all), %.1f s wall on %d "
                      "threads of %s" % (w.n, sample_steps, r.rebuilds - 1, r.rebuilds, t, oracle.num_threads(),
                                         cpu_model())}


def drift_stats(ke, pe, n, dt, every):
    """Energy-drift figures of a sampled series: least-squares slope of E/N in
    epsilon per tau, max |E(t) - E(0)| / |E(0)|, and the RMS fluctuation of E/N."""
    E = (np.asarray(ke) + np.asarray(pe)) / n
    t = np.arange(1, E.size + 1) * every * dt
    slope = float(np.polyfit(t, E, 1)[0]) if E.size > 1 else 0.0
    return {"samples": int(E.size), "slope_per_tau": slope,
            "max_rel_dev": float(np.abs(E - E[0]).max() / abs(E[0])),
            "rms": float(E.std()), "E0_per_particle": float(E[0]), "E_end_per_particle": float(E[-1])}


def timed_steps(ctx, torch, stream, steps, energy_every=0):
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.step(steps, energy_every)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def list_histogram(ctx):
    kp, _ = ctx.get_neighbors()
    cnt = (kp[1:] - kp[:-1]).cpu().numpy()
    pct = np.percentile(cnt, [1, 10, 50, 90, 99]).tolist()
    hist, edges = np.histogram(cnt, bins=np.arange(0, cnt.max() + 11, 10))
    return {"mean": float(cnt.mean()), "std": float(cnt.std()), "min": int(cnt.min()), "max": int(cnt.max()),
            "p1_p10_p50_p90_p99": pct, "bins_of_10": hist.tolist()}


def workload_small(B, torch, args):
    """4000-particle FCC box (10^3 cells, L = 20, T = 1, seed 1): 100 FP64 steps in
    captured graphs, then the 10^4-step energy drift of the FP64 and FP32-mixed paths."""
    from paper_1210_3450_amd import inputs
    w = inputs.small_nve()
    out = {}
    for name, prec in (("fp64", B.MD_PREC_FP64), ("fp32_mixed", B.MD_PREC_FP32_MIXED)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ctx = B.Context(B.make_params(w.n, w.box, precision=prec, flags=B.MD_F_GRAPH), stream=stream)
            ctx.set_state(w.pos, w.vel)
            ctx.step(args.warmup)
            ms = timed_steps(ctx, torch, stream, 100)
            ctx.set_state(w.pos, w.vel)
            ctx.step(args.drift_steps, 10)
            ke, pe = ctx.energy_series()
            st = ctx.stats()
            ctx.close()
        out[name] = {"us_per_step_100": ms * 1e3 / 100, "particle_steps_per_s": w.n * 100 / (ms / 1e3),
                     "drift_%d_steps" % args.drift_steps: drift_stats(ke[:, 0], pe[:, 0], w.n, w.dt, 10),
                     "rebuilds": st["rebuilds"]}
    return {"metric": "particle-steps/s, 4000-particle FCC LJ NVE on 1 MI355X", "value":
            out["fp64"]["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1, "steps": 100,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "fcc4000_rho0.5_rc2.5_skin0.3_dt0.005", "graphs": True}, "paths": out}


def workload_medium(B, torch, args):
    """1,048,576 particles (64^3 FCC cells, L = 128, seed 2): 1000 steps, FP64 and
    FP32-mixed side by side."""
    from paper_1210_3450_amd import inputs
    w = inputs.medium_1m()
    out = {}
    for name, prec in (("fp64", B.MD_PREC_FP64), ("fp32_mixed", B.MD_PREC_FP32_MIXED)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ctx = B.Context(B.make_params(w.n, w.box, precision=prec, flags=B.MD_F_GRAPH), stream=stream)
            ctx.set_state(w.pos, w.vel)
            ctx.autotune(args.tune_cache)
            ctx.step(args.warmup)
            ms = timed_steps(ctx, torch, stream, 1000, 100)
            ke, pe = ctx.energy_series()
            st = ctx.stats()
            ctx.close()
        out[name] = {"ms_per_step": ms / 1000, "particle_steps_per_s": w.n * 1000 / (ms / 1e3),
                     "threads_per_key": st["threads_per_key"], "rebuilds": st["rebuilds"],
                     "drift_1000_steps": drift_stats(ke[:, 0], pe[:, 0], w.n, w.dt, 100)}
    return {"metric": "particle-steps/s, 1M LJ, FP32-mixed vs FP64 on 1 MI355X",
            "value": out["fp32_mixed"]["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
            "steps": 1000, "higher_is_better": True, "dtype": "f32", "dtype_note": MIXED_NOTE, "data": "synthetic",
            "config": {"workload": "fcc1M_rho0.5_rc2.5_skin0.3_dt0.005", "graphs": True}, "paths": out}


def bubble_summary(ctx, torch):
    """md_bubbles at the current state (edge 3, gas below density 0.2), timed."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.bubbles(fields=False)
    dt = time.perf_counter() - t0
    sizes = r["sizes"]
    hist = np.bincount(np.minimum(np.ceil(np.log2(np.maximum(sizes, 1))).astype(int), 20)).tolist() \
        if sizes.size else []
    return {"nbubbles": int(r["nbubbles"]), "gas_subcells": int(r["ngas"]), "largest": int(r["largest"]),
            "subcells": int(np.prod(r["nsub"])), "size_hist_log2": hist, "wall_ms": dt * 1e3}


def pressure_series(ke, vir, V, every, marks):
    """Virial pressure P = (2 KE - W) / (3 V) at the recorded samples."""
    P = (2.0 * ke - vir) / (3.0 * V)
    out = {"every": every, "min": float(P.min()), "step_of_min": int((np.argmin(P) + 1) * every),
           "last": float(P[-1])}
    out["at_step"] = {str(m): float(P[m // every - 1]) for m in marks if 0 < m // every <= P.shape[0]}
    return out


def workload_cavitation(B, torch, args):
    """Cavitation protocol of Sec. IV: 128^3 simple-cubic sites at density 0.7
    (2,097,152 particles, rc = 3.0, seed 4) held at T = 0.9 by a Nose-Hoover
    thermostat (tau = 0.5); all lengths expanded by 1.1 (density 0.526), the
    thermostat switched off, 5000 NVE steps.  Reports the virial pressure before
    and after the expansion and along the NVE run, bubbles (edge-3 subcells,
    gas below density 0.2) at NVE steps 0, 1000 and 5000, list-length
    histograms, drift and throughput of both precisions."""
    from paper_1210_3450_amd import inputs
    w = inputs.cavitation_liquid(n_side=args.cav_side)
    res = {}
    stream = torch.cuda.Stream()
    alpha = 1.1
    with torch.cuda.stream(stream):
        ctx = B.Context(B.make_params(w.n, w.box, rc=w.rc, skin=w.skin, dt=w.dt,
                                      precision=B.MD_PREC_FP32_MIXED, flags=B.MD_F_GRAPH), stream=stream)
        ctx.set_state(w.pos, w.vel)
        t0 = time.time()
        ctx.set_thermostat(w.T, 0.5)
        every = max(1, args.cav_equil // 50)
        ctx.step(args.cav_equil, every)
        ke_s, pe_s = ctx.energy_series()
        vir_s, th_s = ctx.observable_series()
        V0 = w.box[0] ** 3
        H = ke_s[:, 0] + pe_s[:, 0] + th_s[:, 0]
        T_s = 2.0 * ke_s[:, 0] / (3 * w.n - 3)
        half = T_s.shape[0] // 2
        res["equilibration"] = {
            "steps": args.cav_equil, "thermostat": "Nose-Hoover T=%.2f tau=0.5" % w.T,
            "T_mean_second_half": float(T_s[half:].mean()), "T_end": float(T_s[-1]),
            "pressure": pressure_series(ke_s[:, 0], vir_s[:, 0], V0, every, [every, args.cav_equil]),
            "extended_energy_rel_dev": float(np.abs(H - H[0]).max() / abs(H[0])),
            "pe_per_particle_end": float(pe_s[-1, 0] / w.n), "wall_s": time.time() - t0}
        P_liq = float(ctx.pressure()[0])
        ke, _ = ctx.energy()
        ctx.set_thermostat(None, 0.0)
        ctx.rescale_box(alpha)
        ke1, pe1 = ctx.energy()
        P_exp = float(ctx.pressure()[0])
        res["after_expansion"] = {"box": w.box[0] * alpha, "density": w.n / (w.box[0] * alpha) ** 3,
                                  "T": 2.0 * ke1 / (3 * w.n - 3), "pe_per_particle": pe1 / w.n,
                                  "ke_unchanged": bool(abs(ke1 - ke) <= 1e-9 * abs(ke)),
                                  "pressure_before": P_liq, "pressure_after": P_exp}
        p0, v0 = ctx.get_state()
        hist = {"0": list_histogram(ctx)}
        bubbles = {"0": bubble_summary(ctx, torch)}
        V1 = (w.box[0] * alpha) ** 3
        for name, prec in (("fp32_mixed", B.MD_PREC_FP32_MIXED), ("fp64", B.MD_PREC_FP64)):
            c2 = B.Context(B.make_params(w.n, (w.box[0] * alpha,) * 3, rc=w.rc, skin=w.skin, dt=w.dt,
                                         precision=prec, flags=B.MD_F_GRAPH), stream=stream)
            c2.set_state(p0, v0)
            st0 = c2.stats()
            ms1 = timed_steps(c2, torch, stream, 1000, 10)
            if name == "fp32_mixed":
                hist["1000"] = list_histogram(c2)
                bubbles["1000"] = bubble_summary(c2, torch)
            ms2 = timed_steps(c2, torch, stream, args.cav_steps - 1000, 10)
            if name == "fp32_mixed":
                hist[str(args.cav_steps)] = list_histogram(c2)
                bubbles[str(args.cav_steps)] = bubble_summary(c2, torch)
            ke, pe = c2.energy_series()
            vir, _ = c2.observable_series()
            st = c2.stats()
            ke_end, pe_end = c2.energy()
            c2.close()
            res[name] = {"ms_per_step": (ms1 + ms2) / args.cav_steps,
                         "particle_steps_per_s": w.n * args.cav_steps / ((ms1 + ms2) / 1e3),
                         "rebuilds": st["rebuilds"] - st0["rebuilds"], "list_regrows": st["list_regrows"],
                         "drift_%d_steps" % args.cav_steps: drift_stats(ke[:, 0], pe[:, 0], w.n, w.dt, 10),
                         "pressure_nve": pressure_series(ke[:, 0], vir[:, 0], V1, 10,
                                                         [10, 100, 200, 500, 1000, 2000, 3000, 5000]),
                         "T_end": 2.0 * ke_end / (3 * w.n - 3), "pe_per_particle_end": pe_end / w.n}
        ctx.close()
    res["list_length_histograms_nve_step"] = hist
    res["bubbles_nve_step"] = bubbles
    return {"metric": "particle-steps/s, cavitation box (uneven lists), FP32-mixed on 1 MI355X",
            "value": res["fp32_mixed"]["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
            "steps": args.cav_steps, "higher_is_better": True, "dtype": "f32", "dtype_note": MIXED_NOTE,
            "data": "synthetic", "config": {"workload": "sc%d^3_rho0.7_T0.9_rc3.0_expand1.1" % args.cav_side},
            "results": res}


def workload_batch(B, torch, args):
    """256 independent boxes: N_b ~ U{2000..65536}, density ~ U[0.3, 0.8],
    T ~ U[0.7, 1.2] (seed 5), rc = 2.5, FP32-mixed, all advanced together in captured
    graphs after autotuning; baseline: the same boxes one at a time."""
    from paper_1210_3450_amd import inputs
    spec = inputs.batch_spec(args.nbox)
    boxes = [inputs.batch_box(spec, b) for b in range(args.nbox)]
    ntot = int(sum(p.shape[0] for p, _, _ in boxes))
    pos = np.concatenate([p for p, _, _ in boxes])
    vel = np.concatenate([v for _, v, _ in boxes])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        params = [B.make_params(p.shape[0], L, precision=B.MD_PREC_FP32_MIXED, flags=B.MD_F_GRAPH)
                  for p, _, L in boxes]
        ctx = B.Context(params, stream=stream)
        ctx.set_state(pos, vel)
        ctx.autotune(args.tune_cache)
        ctx.step(args.warmup)
        ms = timed_steps(ctx, torch, stream, args.batch_steps, 100)
        ke, pe = ctx.energy_series()
        st = ctx.stats()
        ctx.close()
        # baseline: one box at a time through the single-box path, same kernels
        t_one = 0.0
        n_one = 0
        for k, (p, v, L) in enumerate(boxes[: args.baseline_boxes]):
            c1 = B.Context(B.make_params(p.shape[0], L, precision=B.MD_PREC_FP32_MIXED, flags=B.MD_F_GRAPH),
                           stream=stream)
            c1.set_state(p, v)
            c1.step(5)
            t_one += timed_steps(c1, torch, stream, args.baseline_steps)
            n_one += p.shape[0] * args.baseline_steps
            c1.close()
    drift = [drift_stats(ke[:, b], pe[:, b], boxes[b][0].shape[0], 0.005, 100)["max_rel_dev"]
             for b in range(args.nbox)]
    return {"metric": "particle-steps/s, 256-box LJ ensemble, FP32-mixed on 1 MI355X",
            "value": ntot * args.batch_steps / (ms / 1e3), "unit": "particle-steps/s", "n_gpus": 1,
            "steps": args.batch_steps, "ms_per_step": ms / args.batch_steps, "higher_is_better": True,
            "dtype": "f32", "dtype_note": MIXED_NOTE, "data": "synthetic",
            "config": {"workload": "ensemble%d_N2000-65536_rho0.3-0.8_T0.7-1.2" % args.nbox, "n_particles": ntot,
                       "graphs": True, "threads_per_key": st["threads_per_key"]},
            "one_box_at_a_time": {"particle_steps_per_s": n_one / (t_one / 1e3), "boxes": args.baseline_boxes,
                                  "steps_each": args.baseline_steps},
            "rebuilds": st["rebuilds"], "max_rel_energy_dev_over_boxes": float(max(drift))}


def extra_keys(B, torch, args):
    """Compact figures of the other workloads for the one-line record: the
    4000-particle FP64 box (100 graph steps), the 1M box in both precisions
    (100 steps each) and the 256-box ensemble (autotuned, captured graphs) with
    a one-box-at-a-time baseline on a subset of its boxes."""
    import tempfile
    from paper_1210_3450_amd import inputs
    out = {}
    stream = torch.cuda.Stream()
    # 4000 particles, FP64 and FP32-mixed, captured graphs
    w = inputs.small_nve()
    for name, prec in (("fp64", B.MD_PREC_FP64), ("fp32_mixed", B.MD_PREC_FP32_MIXED)):
        with torch.cuda.stream(stream):
            ctx = B.Context(B.make_params(w.n, w.box, precision=prec, flags=B.MD_F_GRAPH), stream=stream)
            ctx.set_state(w.pos, w.vel)
            ctx.step(20)
            ms = timed_steps(ctx, torch, stream, 100)
            ctx.close()
        out["c1_fcc4000_%s_us_per_step" % name] = ms * 1e3 / 100
    # 1,048,576 particles, both precisions, default layout
    w = inputs.medium_1m()
    for name, prec in (("fp64", B.MD_PREC_FP64), ("fp32_mixed", B.MD_PREC_FP32_MIXED)):
        with torch.cuda.stream(stream):
            ctx = B.Context(B.make_params(w.n, w.box, precision=prec, flags=B.MD_F_GRAPH), stream=stream)
            ctx.set_state(w.pos, w.vel)
            ctx.step(20)
            st0 = ctx.stats()
            ms = timed_steps(ctx, torch, stream, 100)
            st = ctx.stats()
            ctx.close()
        out["c2_fcc1m_%s_ms_per_step" % name] = ms / 100
        out["c2_fcc1m_%s_rebuilds_per_100" % name] = st["rebuilds"] - st0["rebuilds"]
    # 256 boxes of uneven size and density, one context, autotuned
    spec = inputs.batch_spec(256)
    boxes = [inputs.batch_box(spec, b) for b in range(256)]
    ntot = int(sum(p.shape[0] for p, _, _ in boxes))
    pos = np.concatenate([p for p, _, _ in boxes])
    vel = np.concatenate([v for _, v, _ in boxes])
    cache = os.path.join(tempfile.gettempdir(), "mdgpu_bench_tune_%d.txt" % os.getpid())
    with torch.cuda.stream(stream):
        params = [B.make_params(p.shape[0], L, precision=B.MD_PREC_FP32_MIXED, flags=B.MD_F_GRAPH)
                  for p, _, L in boxes]
        ctx = B.Context(params, stream=stream)
        ctx.set_state(pos, vel)
        ke0, pe0 = ctx.batch_energy()
        ctx.autotune(cache)
        ctx.step(20)
        ms = timed_steps(ctx, torch, stream, args.extra_batch_steps)
        st = ctx.stats()
        ctx.close()
        # one box at a time through the single-box path: every 16th box by size
        order = np.argsort(spec.n)
        sub = order[:: max(1, 256 // args.extra_baseline_boxes)][: args.extra_baseline_boxes]
        t_one, n_one = 0.0, 0
        for k in sub:
            p, v, L = boxes[int(k)]
            c1 = B.Context(B.make_params(p.shape[0], L, precision=B.MD_PREC_FP32_MIXED, flags=B.MD_F_GRAPH),
                           stream=stream)
            c1.set_state(p, v)
            c1.step(5)
            t_one += timed_steps(c1, torch, stream, 20)
            n_one += p.shape[0] * 20
            c1.close()
    try:
        os.remove(cache)
    except OSError:
        pass
    E0 = (np.asarray(ke0) + np.asarray(pe0)) / spec.n
    out["c5_ensemble256_ms_per_step"] = ms / args.extra_batch_steps
    out["c5_ensemble256_particle_steps_per_s"] = ntot * args.extra_batch_steps / (ms / 1e3)
    out["c5_one_box_at_a_time_particle_steps_per_s"] = n_one / (t_one / 1e3)
    out["c5_one_box_at_a_time_boxes"] = int(len(sub))
    out["c5_autotuned"] = {"threads_per_key": st["threads_per_key"], "row_tiles": st["row_tiles"],
                           "cell_scale": st["cell_scale"]}
    out["c5_E0_per_particle_min_max"] = [float(E0.min()), float(E0.max())]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncell", type=int, default=200, help="FCC cells per side (200 -> 32M particles)")
    ap.add_argument("--tpk", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fast-rcp", action="store_true",
                    help="skip the FP64 run with the hardware reciprocal and its correction")
    ap.add_argument("--half", action="store_true",
                    help="add the half-list (Newton's third law) runs of both precisions")
    ap.add_argument("--half-steps", type=int, default=100,
                    help="timed steps of each half-list run (about 48 ms per step at 32M)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=25,
                    help="oracle steps of the CPU sample (25 at 32M hold 4 DUTC rebuilds after the initial build)")
    ap.add_argument("--no-extra", action="store_true", help="skip the compact figures of the other workloads")
    ap.add_argument("--no-displacement", action="store_true", help="skip the displacement-rule run")
    ap.add_argument("--extra-batch-steps", type=int, default=100)
    ap.add_argument("--extra-baseline-boxes", type=int, default=16)
    ap.add_argument("--workload", default="fcc32m",
                    choices=["fcc32m", "fcc4000", "fcc1m", "cavitation", "batch256"])
    ap.add_argument("--drift-steps", type=int, default=10000)
    ap.add_argument("--cav-side", type=int, default=128)
    ap.add_argument("--cav-equil", type=int, default=2000)
    ap.add_argument("--cav-steps", type=int, default=5000)
    ap.add_argument("--nbox", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--baseline-boxes", type=int, default=256)
    ap.add_argument("--baseline-steps", type=int, default=100)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--tile", choices=["auto", "on", "off"], default="auto",
                    help="FP32-mixed force pass with LDS-staged partner tiles")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU form "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_3450_amd import binding as B
    from paper_1210_3450_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "fcc32m":
        if args.tune_cache is None:
            import tempfile
            args.tune_cache = os.path.join(tempfile.gettempdir(), "mdgpu_tune_%d.txt" % os.getpid())
        fn = {"fcc4000": workload_small, "fcc1m": workload_medium, "cavitation": workload_cavitation,
              "batch256": workload_batch}[args.workload]
        print(json.dumps(fn(B, torch, args)), flush=True)
        return
    w = inputs.fcc_workload("fcc%d^3_rho0.5" % args.ncell, args.ncell, seed=3, nsteps=args.steps)
    print("bench: %s, N = %d, L = %g, %d warm-up + %d timed steps" % (w.name, w.n, w.box[0], args.warmup,
                                                                       args.steps), file=sys.stderr, flush=True)
    tile_flag = {"auto": 0, "on": B.MD_F_TILE_ON, "off": B.MD_F_TILE_OFF}[args.tile]
    mixed = run_gpu(B, torch, w, B.MD_PREC_FP32_MIXED, args.steps, args.warmup, args.tpk, tile_flag)
    print("bench: FP32-mixed %.3f ms/step" % mixed["ms_per_step"], file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(B, torch, w, B.MD_PREC_FP64, args.steps, args.warmup, args.tpk)
        print("bench: FP64 %.3f ms/step" % fp64["ms_per_step"], file=sys.stderr, flush=True)
    fp64_fast = None
    if not args.no_fp64 and not args.no_fast_rcp:
        fp64_fast = run_gpu(B, torch, w, B.MD_PREC_FP64, args.steps, args.warmup, args.tpk, B.MD_F_FAST_RCP)
        print("bench: FP64 with the corrected hardware reciprocal %.3f ms/step" % fp64_fast["ms_per_step"],
              file=sys.stderr, flush=True)

    disp = None
    if not args.no_displacement:
        disp = run_gpu(B, torch, w, B.MD_PREC_FP32_MIXED, args.steps, args.warmup, args.tpk, tile_flag,
                       B.MD_REBUILD_DISPLACEMENT)
        print("bench: FP32-mixed, displacement rule %.3f ms/step" % disp["ms_per_step"], file=sys.stderr,
              flush=True)

    half = {}
    if args.half:
        for name, prec in (("fp32_mixed", B.MD_PREC_FP32_MIXED), ("fp64", B.MD_PREC_FP64)):
            if prec == B.MD_PREC_FP64 and args.no_fp64:
                continue
            half[name] = run_gpu(B, torch, w, prec, args.half_steps, args.warmup, 0, B.MD_F_HALF_LIST)
            print("bench: half list, %s %.3f ms/step" % (name, half[name]["ms_per_step"]), file=sys.stderr,
                  flush=True)

    rho = 0.5
    rl = w.rc + w.skin
    bpp = algorithmic_bytes_per_particle_step(rho, rl)
    pairs = pairs_within_rc_per_particle(rho, w.rc) * w.n
    force_bytes = bpp * w.n
    achieved = force_bytes / (mixed["force_ms_avg"] / 1e3) / 1e9
    gflops = FLOP_PER_PAIR * pairs / (mixed["ms_per_step"] / 1e3) / 1e9
    interval = args.steps / mixed["rebuilds"] if mixed["rebuilds"] else None  # null in JSON: no rebuild
    step_bpp = bpp + (REBUILD_BYTES_PER_PARTICLE / interval if interval else 0.0)
    step_achieved = step_bpp * w.n / (mixed["ms_per_step"] / 1e3) / 1e9
    traffic = measured_traffic() if args.ncell == 200 else None
    copy_gbs = copy_bandwidth(torch)
    # vector roofline of the force pass: the method's flops (25 per unordered pair within
    # rc) and the FP32 flops the kernel issues (SQ_INSTS_VALU_FLOPS_FP32 + _TRANS per launch,
    # from the committed counter summary) per launch time, against the FP32 vector peak
    alg_tflops = FLOP_PER_PAIR * pairs / (mixed["force_ms_avg"] / 1e3) / 1e12
    issued = summary_value(FLOPS_FILE, "fp32_flops_per_launch") if args.ncell == 200 else None
    issued_tflops = issued / (mixed["force_ms_avg"] / 1e3) / 1e12 if issued else None

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
        "dtype": "f32", "dtype_note": MIXED_NOTE,
        "data": "synthetic: FCC lattice, Maxwell-Boltzmann velocities (seeded)",
        "config": {"workload": "fcc32M_rho0.5_rc2.5_skin0.3_dt0.005" if args.ncell == 200 else w.name,
                   "n_particles": w.n, "box": w.box[0], "rc": w.rc, "skin": w.skin, "dt": w.dt,
                   "precision": "fp32-mixed", "threads_per_key": mixed["threads_per_key"]},
        "gflops": gflops,
        "pair_flop_convention": "25 flop per unordered pair within rc",
        "mixed": mixed,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch from the TCC-to-memory read and write request counters by "
                                     "request size (a plain 1 GiB copy reads exactly 1 GiB and writes 1 GiB by the same "
                                     "rule)",
                     "kernel": "k_force_t<kForceMid> (row tiles staged in LDS: pair forces + kicks + drift)",
                     "bytes_per_particle": bpp, "launch_ms_avg": mixed["force_ms_avg"],
                     "copy_gbs_measured": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "step_roofline": {"bound": "hbm", "achieved": step_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_achieved / HBM_PEAK_GBS, "frac_of_copy": step_achieved / copy_gbs,
                          "bytes_per_particle_step": step_bpp,
                          "rebuild_interval_steps": interval},
        "vector_roofline": {"bound": "alu", "kernel": "k_force_t<kForceMid>", "unit": "TFLOP/s",
                            "peak": FP32_VEC_PEAK_TFLOPS, "algorithmic": alg_tflops,
                            "frac": alg_tflops / FP32_VEC_PEAK_TFLOPS, "issued": issued_tflops,
                            "issued_frac": issued_tflops / FP32_VEC_PEAK_TFLOPS if issued_tflops else None,
                            "convention": "algorithmic: 25 flop per unordered pair within rc; issued: FP32 "
                                          "lane flops counted by SQ_INSTS_VALU_FLOPS_FP32(+_TRANS)"},
    }
    if fp64 is not None:
        f64_tflops = FLOP_PER_PAIR * pairs / (fp64["force_ms_avg"] / 1e3) / 1e12
        out["fp64"] = dict(fp64, gflops=FLOP_PER_PAIR * pairs / (fp64["ms_per_step"] / 1e3) / 1e9,
                           force_achieved_gbs=force_bytes / (fp64["force_ms_avg"] / 1e3) / 1e9,
                           force_hbm_frac=force_bytes / (fp64["force_ms_avg"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                           force_vector_frac=f64_tflops / FP64_VEC_PEAK_TFLOPS,
                           force_algorithmic_tflops=f64_tflops)
    if disp is not None:
        out["mixed_displacement_rule"] = dict(
            disp, rebuild_interval_steps=args.steps / disp["rebuilds"] if disp["rebuilds"] else None,
            note="MD_REBUILD_DISPLACEMENT: rebuild when the largest displacement since the last build "
                 "exceeds skin/2")
    if fp64_fast is not None:
        out["fp64_fast_rcp"] = dict(fp64_fast, gflops=FLOP_PER_PAIR * pairs / (fp64_fast["ms_per_step"] / 1e3) / 1e9,
                                    note="FP64 with 1/r^2 from the hardware reciprocal and the Sec. III.C "
                                         "correction of r^-8 and r^-14")
    if half:
        out["half_list"] = dict(half, note="MD_F_HALF_LIST: each pair once (home cell after the key, 13 forward "
                                           "stencil cells), reactions accumulated per wavefront in LDS and "
                                           "flushed with atomic adds, integration "
                                           "as a separate pass; force_ms_avg covers clearing F, the force pass "
                                           "and the integration pass")
    if not args.no_extra and args.ncell == 200:
        print("bench: other workloads ...", file=sys.stderr, flush=True)
        out.update(extra_keys(B, torch, args))
    if not args.no_cpu:
        print("bench: CPU oracle sample (%d steps) ..." % args.cpu_steps, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
