#!/usr/bin/env python
"""Throughput of the differentiable MLS-MPM hot path on one MI355X.

A bench "step" is one whole trajectory of the hot path on the 3D workload
(64^3 grid, dx = 1/64, 32768 particles on a jittered 32^3 lattice, neo-Hookean
E = 20, nu = 0.3, dt = 5e-4, 256 time steps, full tape): sort + 256 fused
forward launches, mean-height loss and seed, 1 + 256 + 1 reverse launches with
the grid recomputed. Inputs are synthetic and already resident in HBM when the
timed region starts. `value` = particles x time steps x trajectories / seconds
(fwd+bwd particle-steps/s).

Beside it: the roofline figure of the dominant kernel (algorithmic bytes per
launch over its mean duration, HIP events on the launch stream), the FP64 CPU
oracle on a bounded sample of the same workload, the batched 2D workload
(256 scenes in one launch per step) against 256 per-scene runs, and
open-loop controller optimisation iterations of the 3D robot (16 actuators,
30000 particles, 512 steps).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd particle-steps/s, 3D MLS-MPM 64³ grid; batched vs per-scene launches"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_elastic3d.json")
# Launch configurations chosen by the autotuner on MI355X (paper_1910_00935_amd/autotune.py),
# keyed by workload shape and GPU architecture.
TUNED = os.path.join(ROOT, "paper_1910_00935_amd", "tuned.json")


# Sources of the step kernels and their launches (the traffic record is valid
# while these are unchanged).
STEP_SOURCES = ("device_math.h", "mpm.hip", "step_kernels.h", "util_kernels.h")


def _source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1910_00935_amd", "csrc")
    for f in STEP_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_name, knobs):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources with the same launch configuration;
    else None."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_1910_00935_amd.runtime import effective_knobs
    if rec.get("source_hash") != _source_hash() or effective_knobs(rec.get("knobs")) != effective_knobs(knobs):
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("bytes_per_launch")


def tuned_knobs(scene, args, pinned=None):
    """Launch configuration: `pinned` when given, else the autotuner's (a short
    trajectory per candidate, cached per workload shape and GPU), or the library
    defaults with --no-tune."""
    if pinned:
        return dict(pinned)
    if args.no_tune:
        return {}
    from paper_1910_00935_amd import autotune
    return autotune.tune(scene, cache=args.tune_cache, steps=min(scene.steps, 64))


def run_elastic3d(args, torch, rt, scenes):
    sc = scenes.elastic3d()
    T = sc.steps
    N = sc.n_particles
    knobs = tuned_knobs(sc, args, json.loads(args.knobs) if args.knobs else None)
    sim = rt.Simulator.for_scene(sc, knobs=knobs)
    params = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    tape = sim.tape(T, 0)
    final = rt.State.empty(3, N)
    seed = rt.State.empty(3, N)
    grad = rt.State.zeros(3, N)
    gE = torch.zeros(1, device="cuda")

    def step():
        tape.forward(params, init, final)
        sim.loss_mean(final, sc.loss_axis, sc.loss_sign, seed)
        tape.backward(params, seed, grad, gE)

    for _ in range(args.warmup):
        step()
    flags = sim.check_errors()
    if flags:
        raise RuntimeError(f"device error flags {flags}")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    secs = max(wall, gpu_ms / 1e3)
    value = N * T * args.steps / secs

    # Per-kernel durations: the same K trajectories again with every launch of
    # the two step kernels bracketed by HIP events on the launch stream.
    sim.set_knob("timing", 1)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    from paper_1910_00935_amd import _lib as L
    fwd_ms, fwd_n = L.mpm_kernel_stats(sim.ctx, L.MPM_KERNEL_FWD)
    bwd_ms, bwd_n = L.mpm_kernel_stats(sim.ctx, L.MPM_KERNEL_BWD)
    sim.set_knob("timing", 0)
    S = 2 * 3 + 2 * 9
    per = {
        # Algorithmic bytes per launch (particle state only): forward reads
        # state s and writes state s+1 (2 S per particle); reverse reads state
        # s and dL/dstate(s+1) and writes dL/dstate(s) (3 S per particle).
        "k_fwd": {"ms": fwd_ms / max(fwd_n, 1), "launches": fwd_n, "bytes": 2 * S * 4 * N, "total_ms": fwd_ms},
        "k_bwd": {"ms": bwd_ms / max(bwd_n, 1), "launches": bwd_n, "bytes": 3 * S * 4 * N, "total_ms": bwd_ms},
    }
    dom_name = max(per, key=lambda k: per[k]["total_ms"])
    dom = per[dom_name]
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    roofline = {
        "bound": "hbm", "kernel": dom_name + "<3>", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(dom_name, knobs),
        "bytes_per_launch": dom["bytes"], "mean_launch_us": round(dom["ms"] * 1e3, 3),
        "kernels": {k: {"mean_launch_us": round(v["ms"] * 1e3, 3), "launches": v["launches"],
                        "alg_bytes_per_launch": v["bytes"]} for k, v in per.items()},
        # Context for frac: a streaming launch of the same byte count, no dependent work.
        "copy_same_bytes": copy_ceiling(torch, dom["bytes"]),
    }
    # Workgroup wall clocks of one more trajectory (replayed graph, as timed):
    # how much of each launch is workgroup work and how much lies between launches.
    clk = wg_clock_summary(torch, sim, step, rows=2 * T + 8)
    for k, v in clk.items():
        roofline["kernels"][k].update(v)
    return {
        "value": value, "ms_per_step": secs * 1e3 / args.steps, "N": N, "T": T, "roofline": roofline, "knobs": knobs,
        "whole_step_hbm_frac": round((5 * S * 4 * N * T * args.steps / secs) / (HBM_PEAK_GBS * 1e9), 4),
        "gpu_event_ms": gpu_ms, "wall_s": wall,
    }


def wg_clock_summary(torch, sim, run, rows):
    """Runs `run` once with workgroup wall clocks bound and summarises, per step
    kernel, medians over its launches of: the span from the first workgroup's
    start to the last one's end, the median workgroup's duration, and the gap
    from the last workgroup's end to the first start of the next launch of the
    same kernel (consecutive launches only)."""
    import numpy as np
    from paper_1910_00935_amd import _lib as L
    sim.bind_wg_clock(sim.wg_clock_buffer(rows))
    run()
    torch.cuda.synchronize()
    recs = sim.wg_clock()
    sim.bind_wg_clock(None)
    names = {L.MPM_KERNEL_FWD: "k_fwd", L.MPM_KERNEL_BWD: "k_bwd"}
    out = {}
    for kind, name in names.items():
        spans, wgmed, gaps = [], [], []
        for r, (k, st, en) in enumerate(recs):
            if k != kind:
                continue
            spans.append(en.max() - st.min())
            wgmed.append(np.median(en - st))
            if r + 1 < len(recs) and recs[r + 1][0] == kind:
                gaps.append(recs[r + 1][1].min() - en.max())
        if spans:
            out[name] = {"wg_span_us": round(float(np.median(spans)), 3),
                         "wg_median_us": round(float(np.median(wgmed)), 3),
                         "gap_to_next_us": round(float(np.median(gaps)), 3) if gaps else None,
                         "clocked_launches": len(spans)}
    return out


def box_atomics(torch, L, n=64, launches=400):
    """Mean time per launch of the atomic-layout microbenchmark
    (mpm_diag_box_atomics): 128 workgroups adding overlapping 245-node boxes
    of four components into an n^3 grid, back to back on one stream."""
    g = torch.zeros(4 * n ** 3, device="cuda")
    stream = torch.cuda.current_stream()
    names = {0: "node per lane, instruction per component", 1: "lanes over (node, component)",
             2: "plain stores, lanes over (node, component)", 3: "empty launch"}
    out = {}
    for _ in range(3):  # the smallest of three rounds over the layouts
        for layout, name in names.items():
            L.call("mpm_diag_box_atomics", layout, g.data_ptr(), n, 20, stream.cuda_stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            L.call("mpm_diag_box_atomics", layout, g.data_ptr(), n, launches, stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            us = round(e0.elapsed_time(e1) * 1e3 / launches, 3)
            out[name] = min(out.get(name, us), us)
    return out


COPY_MIB = 64  # calibration copy: reads and writes exactly this many MiB


def copy_ceiling(torch, nbytes, launches=200):
    """Mean duration of a plain streaming kernel that reads nbytes/2 and writes
    nbytes/2 (an elementwise scale, back to back on one stream): the HBM
    fraction a launch moving this many bytes reaches with no dependent work."""
    n = max(nbytes // 8, 1)
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(10):
        torch.mul(src, 1.0, out=dst)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(launches):
        torch.mul(src, 1.0, out=dst)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / launches
    gbs = 8 * n / (us * 1e-6) / 1e9
    return {"bytes": 8 * n, "mean_launch_us": round(us, 3), "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def calibration_copy(torch):
    """Kernels of known HBM traffic whose counters give the scale from
    FETCH_SIZE / WRITE_SIZE readings to bytes: a device-to-device copy of
    COPY_MIB MiB (reads and writes COPY_MIB MiB), a fill (writes COPY_MIB MiB)
    and a sum (reads COPY_MIB MiB), each on buffers larger than the caches
    hold after the others ran."""
    n = COPY_MIB * 1024 * 1024 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    other = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    other.fill_(2.0)
    torch.cuda.synchronize()
    s = dst.sum()
    torch.cuda.synchronize()
    return float(s)


CALIBRATION = {"copy": "copyBuffer", "fill": "Fill", "sum": "reduce"}


def _pmc_means(csv_path, counter):
    """Mean value of `counter` per dispatch for each kernel (short name), and
    the largest single reading of each calibration kernel (copy, fill, sum;
    matched by name)."""
    import csv
    sums, counts, cal = {}, {}, {k: 0.0 for k in CALIBRATION}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            name = r["Kernel_Name"]
            for k, pat in CALIBRATION.items():
                if pat in name:
                    cal[k] = max(cal[k], v)
            short = name.split("(")[0].split("::")[-1].split("<")[0]
            sums[short] = sums.get(short, 0.0) + v
            counts[short] = counts.get(short, 0) + 1
    return {k: sums[k] / counts[k] for k in sums}, counts, cal


def summarize_pmc(fetch_csv, write_csv, knobs, command):
    """profiles/traffic_elastic3d.json from a FETCH_SIZE run and a WRITE_SIZE run of
    `bench.py --profile`: per-dispatch KiB of the step kernels, each scaled by
    the ratio of the calibration copy's known size to its own reading."""
    fetch, n_f, cal_f = _pmc_means(fetch_csv, "FETCH_SIZE")
    write, n_w, cal_w = _pmc_means(write_csv, "WRITE_SIZE")
    known_kib = COPY_MIB * 1024.0
    copy_f, copy_w = cal_f["copy"], cal_w["copy"]
    sf = known_kib / copy_f if copy_f > 0 else None
    sw = known_kib / copy_w if copy_w > 0 else None
    kernels = {}
    for k in ("k_fwd", "k_bwd"):
        if k in fetch and k in write and sf and sw:
            rd = fetch[k] * sf * 1024.0
            wr = write[k] * sw * 1024.0
            kernels[k] = {"fetch_kib_raw": fetch[k], "write_kib_raw": write[k], "dispatches": [n_f[k], n_w[k]],
                          "read_bytes": round(rd), "write_bytes": round(wr), "bytes_per_launch": round(rd + wr)}
    rec = {"source_hash": _source_hash(), "knobs": knobs, "command": command,
           "calibration": {"copy_mib": COPY_MIB, "fetch_kib_raw": copy_f, "write_kib_raw": copy_w,
                           "fetch_scale": sf, "write_scale": sw,
                           # Cross-check: the read-only sum and the write-only fill of the same size.
                           "sum_fetch_kib_raw": cal_f["sum"], "fill_write_kib_raw": cal_w["fill"],
                           "sum_fetch_scale": known_kib / cal_f["sum"] if cal_f["sum"] > 0 else None,
                           "fill_write_scale": known_kib / cal_w["fill"] if cal_w["fill"] > 0 else None},
           "kernels": kernels}
    with open(PROFILE_TRAFFIC, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def run_cpu_baseline(sample_steps):
    """The FP64 oracle, single-threaded, on the first `sample_steps` steps of the
    same 3D workload (all 32768 particles): forward, then the reverse pass
    (which recomputes the forward from its checkpoint)."""
    import numpy as np  # noqa: F401
    import oracle as orc
    from paper_1910_00935_amd import scenes
    sc = scenes.elastic3d()
    st = orc.pack(sc.x, sc.v, sc.C, sc.F)
    t0 = time.perf_counter()
    sT, _, _ = orc.run_fwd(sc, sample_steps, st)
    _, seed = orc.loss_mean_pos(sc, sT, sc.loss_axis, sc.loss_sign)
    orc.run_bwd(sc, sample_steps, sample_steps, st, seed)
    dt = time.perf_counter() - t0
    return {"value": sc.n_particles * sample_steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"3D 64^3 workload, all {sc.n_particles} particles, first {sample_steps} of 256 steps, "
                      f"fwd + reverse, {dt:.1f} s", "host": _host()}


def _host():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model}


def run_cpu_baseline_batched(sample_steps, workers):
    """The FP64 oracle on the batched 2D workload with every host core busy:
    the 256 scenes run as independent oracle calls on `workers` threads (the
    oracle is a C library called through ctypes, which releases the GIL),
    first `sample_steps` steps, forward then reverse."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle as orc
    from paper_1910_00935_amd import scenes
    sc = scenes.batched2d()
    parts = [sc.subset([k]) for k in range(sc.n_scenes)]

    def one(s):
        st = orc.pack(s.x, s.v, s.C, s.F)
        sT, _, _ = orc.run_fwd(s, sample_steps, st)
        _, seed = orc.loss_mean_pos(s, sT, s.loss_axis, s.loss_sign)
        orc.run_bwd(s, sample_steps, sample_steps, st, seed)
        return s.n_particles

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        n = sum(ex.map(one, parts))
    dt = time.perf_counter() - t0
    return {"value": n * sample_steps / dt, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"batched 2D workload, all {sc.n_scenes} scenes ({n} particles), first {sample_steps} of "
                      f"{sc.steps} steps, fwd + reverse, one oracle call per scene on {workers} threads, {dt:.1f} s"}


def _median_ms(torch, run, repeats):
    """Median over `repeats` timed calls of run() (after one warmup), each
    bracketed by events on the current stream."""
    import statistics
    run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts), ts


def run_batched(args, torch, rt, scenes, n_scenes=256, steps=256, repeats=5):
    """2D workload of `n_scenes` independent scenes: one context (one launch per
    step for all scenes), the same with the persistent form (one cooperative
    launch per direction), and one context per scene run back to back.
    Medians of `repeats` trajectories each."""
    sc = scenes.batched2d(n_scenes=n_scenes, steps=steps)
    N = sc.n_particles
    knobs = tuned_knobs(sc, args)
    # One configuration for every per-scene run, tuned on a median-size scene.
    counts = [int(sc.offsets[k + 1] - sc.offsets[k]) for k in range(n_scenes)]
    median = sorted(range(n_scenes), key=lambda k: counts[k])[n_scenes // 2]
    knobs_one = tuned_knobs(sc.subset([median]), args)

    def make(s, kn):
        sim = rt.Simulator.for_scene(s, knobs=kn)
        p = rt.params_for_scene(s)
        init = rt.state_for_scene(s)
        tape = sim.tape(steps, 0)
        fin = rt.State.empty(2, s.n_particles)
        seed = rt.State.empty(2, s.n_particles)
        g = rt.State.zeros(2, s.n_particles)
        gE = torch.zeros(s.n_scenes, device="cuda")

        def run():
            tape.forward(p, init, fin)
            sim.loss_mean(fin, s.loss_axis, s.loss_sign, seed)
            tape.backward(p, seed, g, gE)
        return run, sim

    run, sim = make(sc, knobs)
    b_ms, b_all = _median_ms(torch, run, repeats)
    run_p, sim_p = make(sc, {**knobs, "persist": 1})
    p_ms, p_all = _median_ms(torch, run_p, repeats)
    if sim.check_errors() or sim_p.check_errors():
        raise RuntimeError("batched: simulation error flags set")
    per = [make(sc.subset([k]), knobs_one) for k in range(n_scenes)]

    def run_all():
        for r, _ in per:
            r()
    s_ms, s_all = _median_ms(torch, run_all, max(1, repeats // 2))
    # Algorithmic bytes: 5 S per particle-step (S = 48 B in 2D); the grids
    # stay in L2 and are not counted.
    alg = 5 * 48 * N * steps
    return {"workload": f"2D, {n_scenes} scenes x 64^2 grids, {N} particles (log-uniform 500..8000 per scene), "
                        f"{steps} steps, fwd+bwd",
            "batched_particle_steps_per_s": N * steps / (b_ms * 1e-3),
            "persistent_particle_steps_per_s": N * steps / (p_ms * 1e-3),
            "per_scene_particle_steps_per_s": N * steps / (s_ms * 1e-3),
            "speedup": s_ms / b_ms, "batched_ms": round(b_ms, 3), "persistent_ms": round(p_ms, 3),
            "per_scene_ms": round(s_ms, 3),
            "runs_ms": {"batched": [round(t, 3) for t in b_all], "persistent": [round(t, 3) for t in p_all],
                        "per_scene": [round(t, 3) for t in s_all]},
            "hbm_frac": round(alg / (b_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "hbm_frac_persistent": round(alg / (p_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "alg_bytes_per_trajectory": alg,
            "knobs_batched": knobs, "knobs_per_scene": knobs_one}


def run_elastic3d_long(args, torch, rt, scenes, repeats=3):
    """The long 3D workload (128^3 grid, 262144 particles, 1024 steps, tape
    checkpointed every 64 steps, so the reverse pass recomputes each segment
    from its checkpoint): median trajectory time and HBM fraction against
    672 B per particle-step (5 S for the step and its adjoint plus 2 S for the
    segment recompute, S = 96 B)."""
    sc = scenes.elastic3d_long()
    T, N, K = sc.steps, sc.n_particles, sc.ckpt_every
    knobs = tuned_knobs(sc, args)
    sim = rt.Simulator.for_scene(sc, knobs=knobs)
    params = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    tape = sim.tape(T, K)
    final, seed, grad = rt.State.empty(3, N), rt.State.empty(3, N), rt.State.zeros(3, N)
    gE = torch.zeros(1, device="cuda")

    def run():
        tape.forward(params, init, final)
        sim.loss_mean(final, sc.loss_axis, sc.loss_sign, seed)
        tape.backward(params, seed, grad, gE)

    ms, all_ms = _median_ms(torch, run, repeats)
    if sim.check_errors():
        raise RuntimeError("elastic3d_long: simulation error flags set")
    alg = 672 * N * T
    fb = tile_fallback(torch, rt, sc, knobs)
    return {"workload": f"3D, 128^3 grid, {N} particles (64^3 lattice), {T} steps, checkpoints every {K}, fwd+bwd "
                        "with segment recompute",
            "tile_fallback": fb,
            "particle_steps_per_s": N * T / (ms * 1e-3), "ms_per_trajectory": round(ms, 3),
            "runs_ms": [round(t, 3) for t in all_ms], "alg_bytes_per_particle_step": 672,
            "hbm_frac": round(alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4), "knobs": knobs,
            "tape_bytes": tape.nbytes}


def _oracle_rate(sc, steps, act=None):
    """The FP64 oracle's fwd + reverse particle-steps/s on the first `steps`
    steps of a scene (one core) and the seconds it took."""
    import oracle as orc
    st = orc.pack(sc.x, sc.v, sc.C, sc.F)
    t0 = time.perf_counter()
    sT, _, _ = orc.run_fwd(sc, steps, st, act=act)
    _, seed = orc.loss_mean_pos(sc, sT, sc.loss_axis, sc.loss_sign)
    orc.run_bwd(sc, steps, steps, st, seed, act=act)
    dt = time.perf_counter() - t0
    return sc.n_particles * steps / dt, dt


def run_configs(args, torch, rt, scenes, repeats=5):
    """The small 2D workloads' GPU throughput (median trajectory: tape
    forward, loss and seed, reverse pass; the actuated body also its
    actuation signal and adjoint) and the oracle's one-core rate on each,
    and the oracle's rate on a bounded sample of the long 3D workload."""
    import oracle as orc
    out = {}
    for name in ("translate2d", "deform2d", "actuated2d"):
        sc = scenes.make(name) if name in scenes.REGISTRY else getattr(scenes, name)()
        T, N = sc.steps, sc.n_particles
        knobs = tuned_knobs(sc, args)
        sim = rt.Simulator.for_scene(sc, knobs=knobs)
        params = rt.params_for_scene(sc)
        init = rt.state_for_scene(sc)
        tape = sim.tape(T, 0)
        fin, seed, grad = rt.State.empty(2, N), rt.State.empty(2, N), rt.State.zeros(2, N)
        gE = torch.zeros(1, device="cuda")
        act_np = None
        if sc.n_act:
            W = torch.as_tensor(sc.act_W, device="cuda")
            b = torch.as_tensor(sc.act_b, device="cuda")
            gW, gb = torch.zeros_like(W), torch.zeros_like(b)
            gact = torch.zeros(T, sc.n_act, device="cuda")
            act_np = orc.actuation(sc.act_W, sc.act_b, sc.act_omega, sc.dt, T)

        def run():
            if sc.n_act:
                params.act = sim.actuation(W, b, sc.act_omega, T)
                tape.forward(params, init, fin)
                sim.loss_mean(fin, sc.loss_axis, sc.loss_sign, seed)
                tape.backward(params, seed, grad, gE, gact)
                sim.actuation_bwd(W, b, sc.act_omega, T, gact, gW, gb)
            else:
                tape.forward(params, init, fin)
                sim.loss_mean(fin, sc.loss_axis, sc.loss_sign, seed)
                tape.backward(params, seed, grad, gE)

        ms, _ = _median_ms(torch, run, repeats)
        if sim.check_errors():
            raise RuntimeError(f"{name}: simulation error flags set")
        o_steps = T if T <= 64 else 64
        o_rate, o_s = _oracle_rate(sc, o_steps, act=None if act_np is None else act_np[:o_steps])
        out[name] = {"particles": N, "steps": T, "ms_per_trajectory": round(ms, 4),
                     "particle_steps_per_s": N * T / (ms * 1e-3), "knobs": knobs,
                     "hbm_frac": round(5 * 48 * N * T / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 5),
                     "oracle_1core": {"value": o_rate, "sample": f"first {o_steps} steps, {o_s:.2f} s"}}
    sc = scenes.elastic3d_long()
    o_rate, o_s = _oracle_rate(sc, 4)
    out["elastic3d_long_oracle_1core"] = {"value": o_rate, "sample": f"all {sc.n_particles} particles, first 4 "
                                                                     f"steps, fwd + reverse, {o_s:.1f} s"}
    return out


def tile_fallback(torch, rt, sc, knobs, window=64):
    """Fraction of workgroup scatters of the forward pass that fall back to
    global atomics (their stencils' box outgrew the LDS tile), over the first
    and the last `window` steps of the trajectory, with particles sorted once
    at step 0 (as the tape does): forward runs of T - window and T steps,
    the second count minus the first."""
    T = sc.steps
    sim = rt.Simulator.for_scene(sc, knobs={**knobs, "tile_stats": 1})
    act = None
    if sc.n_act:
        W = torch.as_tensor(sc.act_W, device="cuda")
        b = torch.as_tensor(sc.act_b, device="cuda")
        act = sim.actuation(W, b, sc.act_omega, T)
    params = rt.params_for_scene(sc, act=act)
    init = rt.state_for_scene(sc)
    fin = rt.State.empty(sc.dim, sc.n_particles)
    counts = {}
    for n in (window, T - window, T):
        sim.tile_stats()
        tape = sim.tape(n, sc.ckpt_every if sc.ckpt_every and sc.ckpt_every < n else 0)
        tape.forward(params, init, fin)
        counts[n] = sim.tile_stats()
        del tape
    first = counts[window]
    last = tuple(a - b for a, b in zip(counts[T], counts[T - window]))
    frac = lambda c: round(c[1] / max(c[0] + c[1], 1), 4)  # noqa: E731
    return {"window_steps": window, "first": {"lds": first[0], "fallback": first[1], "frac": frac(first)},
            "last": {"lds": last[0], "fallback": last[1], "frac": frac(last)}}


def run_corotated(args, torch, rt, scenes, knobs):
    """The 3D workload with the fixed-corotated stress (polar decomposition in
    every stress evaluation and its hand-written gradient), same launch
    configuration as the headline run."""
    from dataclasses import replace
    sc = replace(scenes.elastic3d(), model=1)
    T, N = sc.steps, sc.n_particles
    sim = rt.Simulator.for_scene(sc, knobs=knobs)
    params = rt.params_for_scene(sc)
    init = rt.state_for_scene(sc)
    tape = sim.tape(T, 0)
    final, seed, grad = rt.State.empty(3, N), rt.State.empty(3, N), rt.State.zeros(3, N)

    def step():
        tape.forward(params, init, final)
        sim.loss_mean(final, sc.loss_axis, sc.loss_sign, seed)
        tape.backward(params, seed, grad)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if sim.check_errors():
        raise RuntimeError("corotated run: simulation error flags set")
    return {"workload": "elastic3d workload with the fixed-corotated stress", "knobs": knobs,
            "particle_steps_per_s": N * T * args.steps / secs, "ms_per_trajectory": secs * 1e3 / args.steps}


def run_robot3d(args, torch, rt, scenes, iters=3, name="robot3d"):
    """The 3D actuated robot (16 actuators, 30000 particles, 512 steps; with
    name="coupled3d", beside 13000 liquid particles): open-loop controller
    optimisation iterations (actuation signal, tape forward, loss, reverse
    replay, actuation adjoint, weight update), timed after one warmup."""
    from paper_1910_00935_amd.controller import OpenLoopController
    sc = scenes.make(name)
    knobs = tuned_knobs(sc, args)
    ctl = OpenLoopController(sc, knobs=knobs)
    hist = [ctl.step(0.05)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        hist.append(ctl.step(0.05))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if ctl.sim.check_errors():
        raise RuntimeError("robot3d: simulation error flags set")
    fb = tile_fallback(torch, rt, sc, knobs)
    what = "3D actuated robot" if name == "robot3d" else "3D actuated robot beside weakly compressible liquid"
    return {"workload": f"{what}, 64^3 grid, {sc.n_particles} particles, {sc.n_act} actuators, "
                        f"{sc.steps} steps; one optimisation iteration = fwd + loss + bwd + weight update",
            "particle_steps_per_s": sc.n_particles * sc.steps * iters / secs,
            "ms_per_iteration": secs * 1e3 / iters, "losses": [round(v, 6) for v in hist], "knobs": knobs,
            "tile_fallback": fb}


def run_smoke(args, torch, rt, scenes, tile=0, repeats=10):
    """The incompressible smoke simulator (Section 4.2, Table 2's workload:
    110^2 periodic grid, 100 steps, 6 Jacobi iterations per projection):
    forward trajectory, loss and seed, reverse pass, timed separately with
    events on the launch stream; medians over `repeats` runs."""
    import statistics
    sc = scenes.smoke()
    sim = rt.SmokeSim.for_scene(sc, tile=tile)
    init = rt.smoke_state(sc)
    target = torch.as_tensor(sc.target, device="cuda")
    seed = torch.empty(3, sc.n, sc.n, device="cuda")
    grad = torch.zeros(3, sc.n, sc.n, device="cuda")
    stream = torch.cuda.current_stream()
    fwd, bwd = [], []
    for r in range(repeats + 2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        sim.forward(init)
        sim.loss(target, seed)
        ev[1].record(stream)
        sim.backward(seed, grad)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if r >= 2:
            fwd.append(ev[0].elapsed_time(ev[1]))
            bwd.append(ev[1].elapsed_time(ev[2]))
    if sim.check_errors():
        raise RuntimeError("smoke: error flags set")
    f, b = statistics.median(fwd), statistics.median(bwd)
    cells = sc.n * sc.n * sc.steps
    state = 3 * sc.n * sc.n * 4
    return {"workload": f"incompressible smoke, {sc.n}^2 periodic grid, {sc.steps} steps, {sc.iters} Jacobi "
                        f"iterations per projection, loss = sum (s_T - target)^2, gradient w.r.t. the initial state",
            "fwd_ms": round(f, 4), "bwd_ms": round(b, 4), "total_ms": round(f + b, 4),
            "cell_steps_per_s": cells / ((f + b) * 1e-3),
            # Per launch: forward reads state s and writes state s+1; reverse
            # reads states s, s+1 and the adjoint of s+1 and writes the adjoint of s.
            "alg_bytes_per_launch": {"fwd": 2 * state, "bwd": 4 * state},
            "launch_us": {"fwd": round(f * 1e3 / sc.steps, 3), "bwd": round(b * 1e3 / sc.steps, 3)},
            "tile": tile or 16, "runs": repeats}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample-steps", type=int, default=128)
    ap.add_argument("--cpu-batched-steps", type=int, default=256)
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-robot", action="store_true")
    ap.add_argument("--no-smoke", action="store_true")
    ap.add_argument("--no-long", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch configuration")
    ap.add_argument("--tune-cache", default=TUNED,
                    help="autotuner results (committed; shapes missing from it are tuned on the spot and added)")
    ap.add_argument("--knobs", default=None, help='launch configuration for the 3D workload as JSON, e.g. \'{"block": 256}\'')
    ap.add_argument("--profile", action="store_true",
                    help="3D workload only, then one calibration copy (for rocprofv3 counter runs)")
    ap.add_argument("--profile-smoke", action="store_true",
                    help="smoke workload only (--steps trajectories), for rocprofv3 runs")
    ap.add_argument("--profile-batched", action="store_true",
                    help="batched 2D workload only (--steps trajectories), then one calibration copy")
    ap.add_argument("--profile-atomics", action="store_true",
                    help="atomic-layout microbenchmark of the scatter-tile flush pattern (one JSON line)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic record from two rocprofv3 --pmc runs of --profile")
    ap.add_argument("--pmc-command", default="", help="command recorded with --summarize-pmc")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, json.loads(args.knobs) if args.knobs else {}, args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the simulator runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1910_00935_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1910_00935_amd import build
        build.build()
    from paper_1910_00935_amd import runtime as rt
    from paper_1910_00935_amd import scenes
    torch.cuda.set_device(0)
    if args.profile_atomics:
        print(json.dumps({"profile": "box_atomics", "us_per_launch": box_atomics(torch, _lib)}), flush=True)
        return
    if args.profile_smoke:
        # The smoke workload's forward, loss and reverse, --steps times, for rocprofv3 runs.
        sc = scenes.smoke()
        sim = rt.SmokeSim.for_scene(sc)
        init = rt.smoke_state(sc)
        target = torch.as_tensor(sc.target, device="cuda")
        seed = torch.empty(3, sc.n, sc.n, device="cuda")
        grad = torch.zeros(3, sc.n, sc.n, device="cuda")
        for _ in range(args.steps):
            sim.forward(init)
            sim.loss(target, seed)
            sim.backward(seed, grad)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "smoke", "flags": sim.check_errors()}), flush=True)
        return
    if args.profile_batched:
        # One batched 2D trajectory (fwd + loss + bwd) per step, for rocprofv3 runs.
        sc = scenes.batched2d()
        knobs = tuned_knobs(sc, args, json.loads(args.knobs) if args.knobs else None)
        sim = rt.Simulator.for_scene(sc, knobs=knobs)
        p = rt.params_for_scene(sc)
        init = rt.state_for_scene(sc)
        tape = sim.tape(sc.steps, 0)
        fin = rt.State.empty(2, sc.n_particles)
        seed = rt.State.empty(2, sc.n_particles)
        g = rt.State.zeros(2, sc.n_particles)
        gE = torch.zeros(sc.n_scenes, device="cuda")
        for _ in range(args.steps):
            tape.forward(p, init, fin)
            sim.loss_mean(fin, sc.loss_axis, sc.loss_sign, seed)
            tape.backward(p, seed, g, gE)
        torch.cuda.synchronize()
        calibration_copy(torch)
        print(json.dumps({"profile": "batched 2D", "knobs": knobs, "flags": sim.check_errors()}), flush=True)
        return
    print("[bench] 3D workload", flush=True)
    elastic3d = run_elastic3d(args, torch, rt, scenes)
    out = {
        "metric": METRIC, "value": round(elastic3d["value"], 1), "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elastic3d["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D MLS-MPM fwd+bwd: 64^3 grid, dx=1/64, 32768 particles (jittered 32^3 lattice "
                               "spaced dx/2), neo-Hookean E=20 nu=0.3, dt=5e-4, 256 steps, full tape, "
                               "loss = mean final height; one bench step = one trajectory",
                   "particles": elastic3d["N"], "time_steps": elastic3d["T"]},
        "roofline": elastic3d["roofline"],
        "whole_step_hbm_frac": elastic3d["whole_step_hbm_frac"],
    }
    out["config"]["knobs"] = elastic3d["knobs"]
    if args.profile:
        calibration_copy(torch)
        print(json.dumps(out), flush=True)
        return
    if not args.no_batched:
        print("[bench] batched 2D workload", flush=True)
        out["batched"] = run_batched(args, torch, rt, scenes)
    if not args.no_configs:
        print("[bench] 2D workloads", flush=True)
        out["configs"] = run_configs(args, torch, rt, scenes)
    if not args.no_long:
        print("[bench] long 3D workload", flush=True)
        out["elastic3d_long"] = run_elastic3d_long(args, torch, rt, scenes)
    if not args.no_robot:
        print("[bench] 3D robot controller optimisation", flush=True)
        out["robot3d"] = run_robot3d(args, torch, rt, scenes)
        print("[bench] 3D robot and liquid controller optimisation", flush=True)
        out["coupled3d"] = run_robot3d(args, torch, rt, scenes, name="coupled3d")
        print("[bench] fixed-corotated model", flush=True)
        out["elastic3d_corotated"] = run_corotated(args, torch, rt, scenes, elastic3d["knobs"])
    if not args.no_smoke:
        print("[bench] smoke simulator", flush=True)
        out["smoke"] = run_smoke(args, torch, rt, scenes)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", flush=True)
        out["cpu_baseline"] = run_cpu_baseline(args.cpu_sample_steps)
        out["cpu_baseline_batched_all_cores"] = run_cpu_baseline_batched(args.cpu_batched_steps, args.cpu_workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
