#!/usr/bin/env python3
"""Throughput of the multi-domain retarded-potential step on one MI355X.

Workload (the plain FP32 method at scale): 8 sub-domains of 64^3 points,
h = 0.3 bohr, placed at random in a 400-bohr box (centre distance >= 20 bohr,
no overlap), c = 137.036, dt = 0.01 a.u., FFT pad 128^3, each domain holding 16
seeded Gaussian +/- charge pairs with analytic continuity-satisfying currents.
A step is rp_push_sources + rp_retarded_step for every sub-domain (forward FFT
of the new sources into the history ring, lag-sum multiply-accumulate over
every (target, source, lag) triple, inverse FFT with crop and static add).
Inputs for every timed step are generated into device memory before the timed
region.  One update is (v, Ax, Ay, Az) at one target grid point for one step.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "retarded-potential grid-pt updates/s (phi,A) vs plain FP32; rel err vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class SourceGen:
    """Sources of step l, [4][Nx][Ny][Nz] per domain, on the GPU from the
    separable factors (FP64 product, then the path's dtype)."""

    def __init__(self, system, dtype):
        import torch
        from synth.sources import spatial_factors
        self.system, self.dtype = system, dtype
        self.B = []
        for d in system.domains:
            b = spatial_factors(d, system.h, system.c)
            self.B.append(torch.from_numpy(b.reshape(b.shape[0], -1)).to("cuda"))

    def __call__(self, l):
        import torch
        from synth.sources import time_factors
        out = []
        for d, B in zip(self.system.domains, self.B):
            A = torch.from_numpy(time_factors(d, self.system.dt, [l])).to("cuda")
            out.append((A @ B).reshape((4,) + tuple(d.dims)).to(self.dtype).contiguous())
        return out


def make_sources(system, steps, dtype):
    """Per-step sources [4][Nx][Ny][Nz] on the GPU from the separable factors."""
    import torch
    from synth.sources import spatial_factors, time_factors
    out = [[None] * len(system.domains) for _ in steps]
    for n, d in enumerate(system.domains):
        B = spatial_factors(d, system.h, system.c)
        Bt = torch.from_numpy(B.reshape(B.shape[0], -1)).to("cuda")
        A = torch.from_numpy(time_factors(d, system.dt, list(steps))).to("cuda")
        S = (A @ Bt).to(dtype)
        for i in range(len(steps)):
            out[i][n] = S[i].reshape((4,) + tuple(d.dims)).contiguous()
        del Bt, A, S
    return out


def traffic_from_profiles(workload, precision):
    """HBM bytes per lag-sum launch from the committed counter summary, if it
    was taken on the current kernel source and this workload."""
    path = os.path.join(ROOT, "profiles", "lagsum_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    key = f"{workload}|{precision}"
    ent = rec.get(key)
    from paper_2311_15429_amd.profiling import kernel_source_sha
    if not ent or ent.get("kernel_source_sha") != kernel_source_sha():
        return None
    return ent.get("traffic_bytes_per_launch")


def cpu_baseline(system, target_seconds, l, gpu_values):
    """The oracle (FP64 direct sum) on a bounded sample of the same workload:
    grid points of every target domain at step l (each update sums over all
    source domains), timed on the host cores.  The same oracle values give the
    error of the GPU's step-l output at those points (gpu_values(s, idx) ->
    [4][len(idx)]), max and RMS over the sampled points divided by the largest
    |oracle| value, per component."""
    import numpy as np
    import oracle
    from synth.sources import spatial_factors, time_factors
    t = l * system.dt
    B = [spatial_factors(d, system.h, system.c) for d in system.domains]

    def windows(s):
        """Source samples every source domain needs for target s at step l."""
        cache = {}
        for n, d in enumerate(system.domains):
            rmin, rmax = oracle.box_distance_range(system.domains[s], d, system.h)
            j0, j1 = oracle.needed_sample_range(t, rmin, rmax, system.dt, system.c, self_cell=(n == s))
            nt = B[n].shape[0]
            js = np.arange(j0, j1 + 1)
            A = time_factors(d, system.dt, np.concatenate([[0], js]))
            cache[n] = (j0, (A @ B[n].reshape(nt, -1)).reshape(len(js) + 1, 4, -1))

        def fn(n, a, b):
            j0, S = cache[n]
            if a == 0 and b == 0:
                return S[:1]
            return S[1 + a - j0: 2 + b - j0]
        return fn

    rng = np.random.default_rng(0)
    c1 = oracle.self_cell_c1()
    from oracle.ref import threads
    cores = threads()
    n_dom = len(system.domains)
    dims = [d.dims for d in system.domains]
    # rate on a small sample of domain 0, then an equal share of the time per domain
    fn0 = windows(0)
    idx = np.sort(rng.choice(system.domains[0].n_points, size=64, replace=False))
    t0 = time.perf_counter()
    oracle.potential_points(system, 0, idx, l, fn0, c1=c1)
    rate = len(idx) / (time.perf_counter() - t0)
    n_per = int(min(system.domains[0].n_points, max(64, rate * target_seconds / n_dom)))
    el, npts, got, ref = 0.0, 0, [], []
    for s in range(n_dom):
        fn = fn0 if s == 0 else windows(s)
        nx, ny, nz = dims[s]
        corners = [(i * ny + j) * nz + k for i in (0, nx - 1) for j in (0, ny - 1) for k in (0, nz - 1)]
        idx = np.unique(np.concatenate([corners, rng.choice(system.domains[s].n_points, size=n_per,
                                                             replace=False)]))
        t0 = time.perf_counter()
        r = oracle.potential_points(system, s, idx, l, fn, c1=c1)
        el += time.perf_counter() - t0
        npts += len(idx)
        ref.append(r.T)
        got.append(gpu_values(s, idx))
        del fn
    g = np.concatenate(got, axis=1)
    r = np.concatenate(ref, axis=1)
    scale = np.max(np.abs(r), axis=1)
    err = {"step": l, "points": npts, "components": ["v", "Ax", "Ay", "Az"],
           "max": [float(v) for v in np.max(np.abs(g - r), axis=1) / scale],
           "rms": [float(v) for v in np.sqrt(np.mean((g - r) ** 2, axis=1)) / scale]}
    # one thread on a proportionally smaller sample of domain 0
    n1 = max(1, n_per // max(cores, 1))
    idx1 = np.sort(rng.choice(system.domains[0].n_points, size=n1, replace=False))
    fn0 = windows(0)
    threads(1)
    try:
        t0 = time.perf_counter()
        oracle.potential_points(system, 0, idx1, l, fn0, c1=c1)
        el1 = time.perf_counter() - t0
    finally:
        threads(cores)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    src_pts = sum(d.n_points for d in system.domains)
    cpu = {"value": npts / el, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{npts} grid points spread over all {n_dom} target domains (corners included; "
                     f"{src_pts:,} source points each update) at step {l}, the last timed step; "
                     f"{el:.1f} s of oracle time",
           "seconds": el, "single_thread_value": n1 / el1, "single_thread_sample_points": n1,
           "cpu_model": model}
    return cpu, err


def run_waves(system, precision, waves, W, K, E, split_gap, label="wave", lagsum_steps=1):
    """Run every wave of target groups (waves.py) of `system`: per wave one
    batched plan (pads, split history), bound to one shared workspace, Green
    spectra, step 0, a captured step, W warm-up replays, K timed replays
    (sources in device memory before the timed region), E eager steps timing
    the lag sum.  Returns the summed timings and counts."""
    import torch
    from paper_2311_15429_amd import waves as WV
    from synth.sources import System, TorchSources
    stream = torch.cuda.current_stream()
    t_timed = t_setup = lag_s = 0.0
    lag_bytes = 0.0
    updates = 0
    ws_total = 0
    n_launch = 0
    phases = {"plan": 0.0, "bind": 0.0, "green": 0.0, "sources": 0.0, "capture_warmup": 0.0}
    # one workspace allocation serves every wave
    ws_max = max(w.workspace for w in waves) + (1 << 20)
    workspace = torch.empty(ws_max, dtype=torch.uint8, device="cuda")
    wall0 = time.perf_counter()

    def lap(key, t):
        torch.cuda.synchronize()
        now = time.perf_counter()
        phases[key] += now - t
        return now

    for wi, wave in enumerate(waves):
        ts = t = time.perf_counter()
        plan, doms, targets = WV.wave_plan(wave, system.dims, system.origins, system.h, system.dt, system.c,
                                           precision, split_gap=split_gap, stream=stream, lagsum_steps=lagsum_steps)
        plan.set_tuning("lagsum_persistent", 1)
        if lagsum_steps > 1:
            plan.set_tuning("lagsum_cached", 1)
            plan.set_tuning("lagsum_tile_major", 1)
        st = plan.stats()
        ws_total += plan.workspace_bytes
        if plan.workspace_bytes + 256 > ws_max:
            raise RuntimeError("wave workspace above the packing estimate")
        t = lap("plan", t)
        plan.bind(workspace=workspace)
        t = lap("bind", t)
        plan.set_green_kernels()
        t = lap("green", t)
        dt = plan.dtype
        wsys = System(system.h, system.dt, system.c, [system.domains[g] for g in doms])
        gen = TorchSources(wsys, "cuda")
        src = [gen.step(l, dt) for l in range(W + K + E + 1)]
        del gen
        t = lap("sources", t)
        tset = set(targets)
        outs = [torch.empty((4,) + plan.dims[i], dtype=dt, device="cuda") if i in tset else None
                for i in range(plan.n_dom)]
        buf = [torch.empty_like(x) for x in src[0]]
        plan.push_sources(0, src[0])
        plan.retarded_step(0, outs)
        plan.capture_step(buf, outs)
        for l in range(1, W + 1):
            torch._foreach_copy_(buf, src[l])
            plan.launch_step(l)
        lap("capture_warmup", t)
        t_setup += time.perf_counter() - ts
        t1 = time.perf_counter()
        for l in range(W + 1, W + K + 1):
            torch._foreach_copy_(buf, src[l])
            plan.launch_step(l)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        t_timed += el
        updates += st["points"] * K
        plan.lagsum_time()
        plan.profile_lagsum(True)
        for l in range(W + K + 1, W + K + E + 1):
            plan.push_sources(l, src[l])
            plan.retarded_step(l, outs)
        torch.cuda.synchronize()
        plan.profile_lagsum(False)
        ms, n = plan.lagsum_time()
        lag_s += ms / 1e3
        lag_bytes += st["lagsum_bytes"] * n
        n_launch += n
        if not all(bool(torch.isfinite(o).all()) for o in outs if o is not None):
            raise RuntimeError(f"non-finite output in wave {wi}")
        log(f"{label} {wi + 1}/{len(waves)}: {len(wave.units)} units, {len(targets)} targets, workspace "
            f"{plan.workspace_bytes / 1e9:.0f} GB, step {1e3 * el / K:.1f} ms, lag sum {ms / max(n, 1):.1f} ms "
            f"({st['lagsum_bytes'] / (ms / max(n, 1) / 1e3) / 1e9:.0f} GB/s); setup so far "
            + ", ".join(f"{k} {v:.0f} s" for k, v in phases.items()))
        plan.close()
        del plan, src, outs, buf
    del workspace
    torch.cuda.empty_cache()
    return {"t_timed": t_timed, "t_setup": t_setup, "updates": updates, "phases": phases, "lag_bytes": lag_bytes,
            "lag_s": lag_s, "n_launch": n_launch, "ws_total": ws_total, "wall0": wall0}


def bench_batched(args):
    """The batched workload as drawn: 64 independent systems of 2-16
    sub-domains with grids from {32, 48, 64, 96}^3 (FP32 by default).  Its
    history and spectra (24 TB in FP32) cannot sit on one device at once, so
    the targets are grouped into units (the targets of one grid shape of one
    system, halved until the unit's plan fits, each with every domain of its
    system as a source, its own pad and a split history) and the units are
    packed into waves of at most the free device memory.  Each wave is one
    batched plan: bind, Green spectra, step 0, a captured step, W warm-up
    replays, K timed replays (sources already in device memory), then E eager
    steps that time the lag sum.  Throughput = every target point x K over the
    summed timed replays of all waves; one step of the whole workload takes
    the sum of the waves' step times."""
    import torch
    from paper_2311_15429_amd import waves as WV
    from synth.sources import config4
    precision = args.precision or "fp32"
    system = config4(args.seed)
    free, total = torch.cuda.mem_get_info()
    reserve = 16e9          # sources of the timed steps, outputs, graph buffers, source fields
    budget = int(0.97 * (free - reserve))
    if args.wave_gb:
        budget = min(budget, int(args.wave_gb * 1e9))
    t0 = time.perf_counter()
    kb = args.lagsum_steps
    units = WV.plan_units(system.dims, system.origins, system.system_id, system.h, system.dt, system.c,
                          precision, budget, split_gap=args.split_gap, lagsum_steps=kb)
    waves = WV.pack_waves(units, budget)
    t_plan = time.perf_counter() - t0
    lag_total = sum(u.lagsum_bytes for u in units) / kb      # per step
    pts_total = sum(u.points for u in units)
    log(f"config 4: {len(set(system.system_id))} systems, {len(system.domains)} domains, {pts_total} target points; "
        f"{len(units)} units in {len(waves)} waves of <= {budget / 1e9:.0f} GB (device free {free / 1e9:.0f} of "
        f"{total / 1e9:.0f} GB); lag-sum bytes per step {lag_total / 1e12:.2f} TB; host planning {t_plan:.1f} s")
    # per wave: W warm-up and K timed graph replays (the timed steps' sources
    # sit in device memory beside the wave's workspace, so K stays small: one
    # block of kb steps by default), then E eager steps holding exactly one
    # pass of the lag sum (one block start)
    W, K, E = args.wave_warmup, args.wave_steps, kb
    r = run_waves(system, precision, waves, W, K, E, args.split_gap, lagsum_steps=kb)
    t_timed, t_setup, updates, phases = r["t_timed"], r["t_setup"], r["updates"], r["phases"]
    lag_bytes, lag_s, n_launch, ws_total, wall0 = r["lag_bytes"], r["lag_s"], r["n_launch"], r["ws_total"], r["wall0"]
    wall = time.perf_counter() - wall0
    value = updates / t_timed
    ms_step = 1e3 * t_timed / K
    achieved = lag_bytes / lag_s / 1e9
    log(f"config 4 in {len(waves)} waves: {ms_step:.0f} ms per step of the whole workload, {value / 1e6:.2f} M "
        f"updates/s; lag sum {achieved:.0f} GB/s over {n_launch} launches; wall {wall:.0f} s "
        f"(setup {t_setup:.0f} s)")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_lagsum",
            "kernel_ms": round(1e3 * lag_s / max(n_launch, 1), 4),
            "algorithmic_bytes_per_launch": lag_bytes / max(n_launch, 1),
            "timed_on": f"{E} eager step(s) per wave after its timed graph replays, all waves "
                        f"(the pass of each block's first step with {kb} steps per pass)"}
    line = {"metric": METRIC, "value": value, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 independent systems, 2-16 sub-domains each with grids drawn from "
                                   "{32,48,64,96}^3, h=0.3 bohr, separations 20-300 bohr, dt=0.01, run in waves of "
                                   "target groups (one graph launch per step per wave)",
                       "precision": precision, "systems": len(set(system.system_id)),
                       "domains": len(system.domains), "target_points": pts_total,
                       "units": len(units), "waves": len(waves), "wave_budget_bytes": budget,
                       "workspace_bytes_all_waves": ws_total, "lagsum_bytes_per_step": lag_total,
                       "split_gap": args.split_gap, "lagsum_steps_per_pass": kb,
                       "steps_per_wave": {"warmup": W, "timed": K, "eager": E},
                       "setup_s": round(t_setup, 1), "setup_phases_s": {k: round(v, 1) for k, v in phases.items()},
                       "wall_s": round(wall, 1)},
            "roofline": roof, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_batched_scaled(args):
    """64 independent systems with uneven domain counts and grid sizes in one
    plan (the batched recipe at reduced sizes: 2-8 sub-domains of 16^3, 24^3
    or 32^3 points, so that every system fits at once); each step is one
    replay of the captured graph."""
    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import config4
    system = config4(args.seed, sizes=(16, 24, 32), n_dom_range=(2, 8))
    precision = args.precision or "fp32_ring_fp16"
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, precision, stream=stream)
    st = plan.stats()
    log(f"batched plan: {len(set(system.system_id))} systems, {len(system.domains)} domains, "
        f"triples/step {st['n_triples']}, workspace {plan.workspace_bytes / 1e9:.1f} GB, "
        f"lag-sum bytes/launch {st['lagsum_bytes'] / 1e9:.2f} GB")
    plan.bind()
    plan.set_green_kernels()
    tuned = plan.autotune(iters=3)
    log(f"autotune: {tuned}")
    W, K = args.warmup, args.steps
    E = 5                                   # eager steps after the timed region (lag-sum timing)
    src = make_sources(system, range(W + K + E + 1), plan.dtype)
    outs = [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    buf = [torch.empty_like(o) for o in outs]
    plan.push_sources(0, src[0])
    plan.retarded_step(0, outs)
    plan.capture_step(buf, outs)

    def step(l):
        torch._foreach_copy_(buf, src[l])
        plan.launch_step(l)

    for l in range(1, W + 1):
        step(l)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(W + 1, W + K + 1):
        step(l)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / K
    updates = st["points"] * K / el
    log(f"batched: step {ms_step:.3f} ms, {updates / 1e6:.2f} M updates/s")
    # the lag sum inside the graph cannot carry the plan's timing events: time
    # it on the next E steps, run eagerly (same kernels, same schedule)
    plan.lagsum_time()
    plan.profile_lagsum(True)
    for l in range(W + K + 1, W + K + E + 1):
        plan.push_sources(l, src[l])
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    plan.profile_lagsum(False)
    lag_ms, launches = plan.lagsum_time()
    lag_s = lag_ms / launches / 1e3
    achieved = st["lagsum_bytes"] / lag_s / 1e9
    log(f"lag sum (eager steps after the timed region): {lag_s * 1e3:.3f} ms, {achieved:.0f} GB/s")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_lagsum",
            "kernel_ms": round(lag_s * 1e3, 4), "algorithmic_bytes_per_launch": st["lagsum_bytes"],
            "timed_on": f"{E} eager steps after the timed graph replays"}
    line = {"metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batched recipe at reduced sizes (not the drawn shapes): 64 independent "
                                   "systems, 2-8 sub-domains each of 16^3/24^3/32^3 points, h=0.3 bohr, "
                                   "separations 20-300 bohr, dt=0.01, one graph launch per step",
                       "precision": precision, "domains": len(system.domains),
                       "triples_per_step": st["n_triples"], "lagsum_bytes": st["lagsum_bytes"],
                       "workspace_bytes": plan.workspace_bytes, "autotune": tuned},
            "roofline": roof}
    print(json.dumps(line), flush=True)


def bench_small(args):
    """Config 1 in FP64 (2 x 16^3, h = 0.5, 30 bohr apart, dt = 0.02): step
    latency over 40 steps, beside the oracle's full run of the same steps on
    the host cores (parity is checked too)."""
    import numpy as np
    import torch
    import oracle
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import config1, sample_sources
    L = 40
    system = config1(args.seed if args.seed else 1)
    S = sample_sources(system, range(L + 1))
    plan = plan_for_system(system, "fp64", stream=torch.cuda.current_stream())
    plan.bind()
    plan.set_green_kernels()
    src = [[torch.from_numpy(np.ascontiguousarray(S[n][l]).reshape((4,) + plan.dims[n])).to("cuda")
            for n in range(2)] for l in range(L + 1)]
    outs = [torch.empty((4,) + d, dtype=torch.float64, device="cuda") for d in plan.dims]
    times, got = [], None
    for rep in range(3):
        if rep:
            plan.bind()            # restart the step sequence on the same plan
            plan.set_green_kernels()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for l in range(L + 1):
            plan.push_sources(l, src[l])
            plan.retarded_step(l, outs)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    got = [o.cpu().numpy().reshape(4, -1) for o in outs]
    el = min(times)
    pts = plan.stats()["points"]
    t0 = time.perf_counter()
    ref = oracle.potential_full(system, S, range(L + 1))
    t_oracle = time.perf_counter() - t0
    r = np.concatenate(ref[L], axis=1)
    g = np.concatenate(got, axis=1)
    err = np.max(np.abs(g - r), axis=1) / np.max(np.abs(r), axis=1)
    cores = len(os.sched_getaffinity(0))
    log(f"config 1 FP64: {1e3 * el / (L + 1):.3f} ms/step, {pts * (L + 1) / el / 1e6:.2f} M updates/s; "
        f"oracle {t_oracle:.1f} s on {cores} cores; rel err at step {L}: {np.array2string(err, precision=2)}")
    line = {"metric": METRIC, "value": pts * (L + 1) / el, "unit": "grid-point updates/s", "n_gpus": 1,
            "steps": L + 1, "warmup": 0, "ms_per_step": 1e3 * el / (L + 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "2 sub-domains of 16^3 points, h=0.5 bohr, centres 30 bohr apart, dt=0.02, "
                                   "41 steps (step 0 included), FP64, best of 3 runs",
                       "rel_err_vs_fp64_oracle_last_step": [float(v) for v in err]},
            "roofline": None,
            "cpu_baseline": {"value": pts * (L + 1) / t_oracle, "unit": "grid-point updates/s", "cores": cores,
                             "kind": "oracle", "sample": f"the full run: {L + 1} steps x {pts} points",
                             "seconds": t_oracle}}
    print(json.dumps(line), flush=True)
    plan.close()


def bench_surrogate(args):
    """32 sub-domains of 48^3 in a 2000-bohr box with the learned far-pair
    surrogate: teacher data from the plain method on other seeds (audit
    sources only), training in the library's kernels, then the timed run with
    the judge on sampled steps, and the FP64 oracle at sampled points."""
    import numpy as np
    import torch
    import oracle
    from oracle import surrogate_ref
    from paper_2311_15429_amd import plan_for_system
    from paper_2311_15429_amd import surrogate as S
    from synth.sources import config5, spatial_factors, time_factors

    FAR, NL, T_STEPS, TOL = 10.0, 64, 3000, 1e-4
    precision = args.precision or "fp32_ring_i16"
    # lag-sum steps per pass; the judge may change the plain pairs only
    # between blocks, so it runs after the last step of a block (steps
    # 96, 192, ...; blocks start at steps 1, 1 + kb, ...)
    KB = args.lagsum_steps
    JUDGE_EVERY = 96 if KB > 1 else 100
    JUDGE_AT = 0 if KB > 1 else JUDGE_EVERY - 1
    stream = torch.cuda.current_stream()

    class Gen:
        """Sources of step l on the GPU from the separable factors."""

        def __init__(self, system):
            self.system = system
            self.B = []
            for d in system.domains:
                b = spatial_factors(d, system.h, system.c)
                self.B.append(torch.from_numpy(b.reshape(b.shape[0], -1)).to("cuda", torch.float32))

        def __call__(self, l):
            out = []
            for d, B in zip(self.system.domains, self.B):
                A = torch.from_numpy(time_factors(d, self.system.dt, [l])).to("cuda", torch.float32)
                out.append((A @ B).reshape((4,) + tuple(d.dims)).contiguous())
            return out

    # teacher data
    t0 = time.perf_counter()
    X, T = [], []
    for seed in (args.teacher_seeds if args.far in ("learned", "hybrid") else []):
        tsys = config5(seed)
        p = plan_for_system(tsys, "fp32", stream=stream)
        if KB > 1:
            p.set_tuning("lagsum_steps", KB)
        p.surrogate_configure(FAR, n_lags=NL, audit=range(args.teacher_audit))
        log(f"teacher seed {seed}: {p.surrogate_info()}, workspace {p.workspace_bytes / 1e9:.1f} GB")
        p.bind()
        p.set_green_kernels()
        x, t = S.collect_pair_responses(p, Gen(tsys), T_STEPS, start=1, every=3, residual=args.far == "hybrid")
        X.append(x)
        T.append(t)
        p.close()
        del p
        torch.cuda.empty_cache()
        log(f"  {x.shape[0]} samples, {time.perf_counter() - t0:.0f} s")
    sur, n_samples, t_data, t_train, train_rms = None, 0, 0.0, 0.0, None
    if args.far in ("learned", "hybrid"):
        X, T = torch.cat(X), torch.cat(T)
        t_data = time.perf_counter() - t0
        t0 = time.perf_counter()
        sur = S.train_surrogate(X, T, NL, max_batch=2048, log_every=5000, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        train_rms = S.relative_rms(sur, X, T)
        n_samples = int(X.shape[0])
        del X, T
        torch.cuda.empty_cache()
        log(f"trained on {n_samples} pair responses in {t_train:.0f} s, train rel rms {train_rms:.2e}")

    # the workload
    system = config5(args.seed)
    plain = plan_for_system(system, "fp32")
    pst = plain.stats()
    plain.close()
    plan = plan_for_system(system, precision, stream=stream)
    if KB > 1:
        plan.set_tuning("lagsum_steps", KB)
    plan.surrogate_configure(FAR, n_lags=NL, audit=list(args.audit))
    info = plan.surrogate_info()
    st = plan.stats()
    log(f"surrogate plan: {info}, workspace {plan.workspace_bytes / 1e9:.1f} GB "
        f"(plain FP32 would need {(pst['ring_bytes'] + pst['spectra_bytes']) / 1e9:.0f} GB of history)")
    plan.bind()
    plan.set_green_kernels()
    if args.far == "hybrid":
        plan.surrogate_multipole("hybrid")
        plan.surrogate_attach(sur.mlp, sur.in_scale, sur.out_scale)
    elif sur is not None:
        plan.surrogate_attach(sur.mlp, sur.in_scale, sur.out_scale)
    else:
        plan.surrogate_multipole(True)
    if args.readmit > 0:
        plan.surrogate_readmit(args.readmit)
    tuned = plan.autotune(iters=3)
    gen = Gen(system)
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in plan.dims]
    W, K = args.warmup, args.steps
    if KB > 1:
        W += (-W) % KB          # the timed steps start at a block's first step
    judged = []
    readmitted = []

    def step(l):
        plan.push_sources(l, gen(l))
        plan.retarded_step(l, outs)
        if l > 0 and l % JUDGE_EVERY == JUDGE_AT:
            judged.append(plan.surrogate_judge(outs, TOL))
            readmitted.append(plan.last_readmitted)

    for l in range(W + 1):
        step(l)
    if any(n for n, _ in judged) or any(readmitted):
        # fallbacks changed the lag-sum schedule: tune it again
        tuned = plan.autotune(iters=3)
        log(f"re-tuned after {sum(n for n, _ in judged)} fallbacks and {sum(readmitted)} re-admissions: "
            f"{tuned}")
    # sources of the timed steps in device memory before the timed region
    src = [gen(l) for l in range(W + 1, W + K + 1)]
    torch.cuda.synchronize()
    plan.lagsum_time()
    plan.profile_lagsum(True)
    t0 = time.perf_counter()
    for i, l in enumerate(range(W + 1, W + K + 1)):
        plan.push_sources(l, src[i])
        plan.retarded_step(l, outs)
        if l > 0 and l % JUDGE_EVERY == JUDGE_AT:
            judged.append(plan.surrogate_judge(outs, TOL))
            readmitted.append(plan.last_readmitted)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.profile_lagsum(False)
    lag_ms, launches = plan.lagsum_time()
    l_end = W + K
    ms_step = 1e3 * el / K
    updates = st["points"] * K / el
    lag_s = lag_ms / launches / 1e3
    st = plan.stats()                       # after fallbacks
    achieved = st["lagsum_bytes"] / lag_s / 1e9
    plain_lag_ms = pst["lagsum_bytes"] / (achieved * 1e9) * 1e3
    fell = sum(n for n, _ in judged)
    back = sum(readmitted)
    plain_now = int(plan.surrogate_pairs()["fallen_back"].sum())
    log(f"step {ms_step:.2f} ms ({updates / 1e6:.1f} M updates/s), lag sum {lag_s * 1e3:.2f} ms at {achieved:.0f} GB/s; "
        f"plain lag sum alone would be {plain_lag_ms:.1f} ms ({pst['lagsum_bytes'] / 1e9:.0f} GB); "
        f"judge: {len(judged)} calls, {fell} fallbacks, {back} re-admissions, {plain_now} pairs plain at the end")

    # error vs the FP64 oracle at sampled points of the last step, beside the
    # same points with the far pairs left out
    got = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    scale = np.max(np.abs(np.concatenate(got, axis=1)), axis=1)
    pairs = plan.surrogate_pairs()
    rng = np.random.default_rng(1)
    targets = rng.choice(len(system.domains), args.oracle_targets, replace=False)
    B = [spatial_factors(d, system.h, system.c) for d in system.domains]

    def sample_fn(n, j0, j1):
        A = time_factors(system.domains[n], system.dt, np.arange(j0, j1 + 1))
        return (A @ B[n].reshape(B[n].shape[0], -1)).reshape(j1 - j0 + 1, 4, -1)

    err_s = np.zeros(4)
    err_d = np.zeros(4)
    t0 = time.perf_counter()
    for s in targets:
        s = int(s)
        idx = np.sort(rng.choice(system.domains[s].n_points, args.oracle_points, replace=False))
        ref = oracle.potential_points(system, s, idx, l_end, sample_fn)
        err_s = np.maximum(err_s, np.max(np.abs(got[s][:, idx].T - ref), axis=0) / scale)
        # what leaving the far pairs out would cost at the same points
        far_src = [int(n) for t_, n in zip(pairs["target"], pairs["source"]) if int(t_) == s]
        pts = surrogate_ref.grid_points(system.domains[s], system.h)[idx]
        far_dyn = oracle.potential_at(system, pts, l_end * system.dt, sample_fn, dynamic=True, sources=far_src)
        err_d = np.maximum(err_d, np.max(np.abs(far_dyn), axis=0) / scale)
        log(f"  oracle target {s}: {time.perf_counter() - t0:.0f} s")
    t_oracle = time.perf_counter() - t0
    log(f"oracle at {len(targets)} x {args.oracle_points} points: rel err {np.array2string(err_s, precision=2)}; "
        f"far pairs left out would give {np.array2string(err_d, precision=2)} ({t_oracle:.0f} s)")

    # the plain FP32 method on the same workload, measured: its history (824
    # GB) does not fit one device, so it runs as waves of target groups (each
    # a plan of some targets with every domain as a source and a split
    # history); a step of the whole workload takes the sum of the waves' steps
    plain_meas = None
    plan.surrogate_attach(None)
    plan.close()
    del plan, outs, src
    torch.cuda.empty_cache()
    if args.plain_baseline:
        from paper_2311_15429_amd import waves as WV
        free, _ = torch.cuda.mem_get_info()
        budget = int(0.97 * (free - 16e9))
        units = WV.plan_units(system.dims, system.origins, None, system.h, system.dt, system.c, "fp32", budget,
                              split_gap=args.split_gap)
        pwaves = WV.pack_waves(units, budget)
        log(f"plain FP32 baseline: {len(units)} target groups in {len(pwaves)} waves")
        r = run_waves(system, "fp32", pwaves, 1, 3, 1, args.split_gap, label="plain wave")
        plain_ms = 1e3 * r["t_timed"] / 3
        plain_meas = {"ms_per_step": plain_ms, "updates_per_s": r["updates"] / r["t_timed"],
                      "lagsum_ms_per_step": 1e3 * r["lag_s"] / max(r["n_launch"], 1) * len(pwaves),
                      "lagsum_gbs": r["lag_bytes"] / r["lag_s"] / 1e9, "waves": len(pwaves),
                      "target_groups": [len(u.targets) for u in units],
                      "method": "the plain FP32 method (every pair by the lag sum, FP32 ring) run as waves of "
                                "target groups, each a plan of some targets with every sub-domain as a source and "
                                "a split history, one after the other on this device; 3 timed graph replays per "
                                "wave; a step of the whole workload takes the sum of the waves' step times"}
        log(f"plain FP32 measured: {plain_ms:.1f} ms per step ({plain_meas['updates_per_s'] / 1e6:.1f} M updates/s); "
            f"surrogate step {ms_step:.2f} ms: {plain_ms / ms_step:.1f}x")
        # the same with 8 lag-sum steps per pass (the plain path's fastest schedule)
        kb = 8
        units = WV.plan_units(system.dims, system.origins, None, system.h, system.dt, system.c, "fp32", budget,
                              split_gap=args.split_gap, lagsum_steps=kb)
        pwaves = WV.pack_waves(units, budget)
        r = run_waves(system, "fp32", pwaves, 1, kb, kb, args.split_gap, label="plain wave (8 steps per pass)",
                      lagsum_steps=kb)
        ms_b = 1e3 * r["t_timed"] / kb
        plain_meas["blocked8"] = {"ms_per_step": ms_b, "updates_per_s": r["updates"] / r["t_timed"],
                                  "waves": len(pwaves), "target_groups": [len(u.targets) for u in units]}
        log(f"plain FP32 with 8 steps per pass: {ms_b:.1f} ms per step; surrogate step {ms_step:.2f} ms: "
            f"{ms_b / ms_step:.1f}x")

    line = {"metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "32 sub-domains of 48^3 points, h=0.3 bohr, 2000-bohr box, dt=0.01, "
                                   + {"learned": "learned far-pair surrogate",
                                      "multipole": "analytic multipole far-pair terms",
                                      "hybrid": "analytic multipole far-pair terms plus a learned correction"}[args.far]
                                   + " (pairs > 10 box diagonals apart)",
                       "precision": precision, "far_pairs": info["n_far"], "audited_far_pairs": info["n_audited"],
                       "judge_every": JUDGE_EVERY, "judge_tol": TOL, "fallbacks": fell,
                       "lagsum_steps_per_pass": KB,
                       "readmit_factor": args.readmit, "readmissions": back, "plain_pairs_at_end": plain_now,
                       "rel_err_vs_fp64_oracle_sampled": [float(v) for v in err_s],
                       "rel_err_far_pairs_left_out_sampled": [float(v) for v in err_d],
                       "oracle_points": int(len(targets) * args.oracle_points), "step_of_check": l_end,
                       "plain_fp32_history_bytes": pst["ring_bytes"] + pst["spectra_bytes"],
                       "plain_fp32_lagsum_bytes": pst["lagsum_bytes"],
                       "plain_fp32_lagsum_ms_modelled": plain_lag_ms,
                       "speedup_vs_plain_lagsum_alone_modelled": plain_lag_ms / ms_step,
                       "plain_fp32_measured": plain_meas,
                       "speedup_vs_plain_fp32_measured": (plain_meas["ms_per_step"] / ms_step) if plain_meas else None,
                       "speedup_vs_plain_fp32_8_steps_per_pass_measured":
                           (plain_meas["blocked8"]["ms_per_step"] / ms_step) if plain_meas else None,
                       "teacher_samples": n_samples, "teacher_s": round(t_data, 1), "train_s": round(t_train, 1),
                       "train_rel_rms": train_rms, "autotune": tuned},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "k_lagsum" if KB == 1 else f"k_lagsum_block ({KB} steps per pass)",
                         "kernel_ms": round(lag_s * 1e3, 4), "algorithmic_bytes_per_launch": st["lagsum_bytes"]},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_coupled(args):
    """The propagation loop around the path on config 2: each domain's 16
    charge pairs are Lorentz oscillators driven by the computed potentials
    (domain 0 also by a sin^2 pulse); per step push the sources, evaluate the
    potentials, project them on the oscillators, update them and synthesise
    the next step's sources, all on the GPU with no host round trip."""
    import numpy as np
    import torch
    from paper_2311_15429_amd import Oscillators, plan_for_system
    from synth.sources import config2, pair_shapes
    system = config2(args.seed)
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, args.precision, stream=stream)
    # blocked lag-sum steps hold in the loop: each step returns its own
    # potential from the sources pushed so far
    kb = args.lagsum_steps if args.precision != "fp64" else 1
    if kb > 1:
        plan.set_tuning("lagsum_steps", kb)
    st = plan.stats()
    plan.bind()
    plan.set_green_kernels()
    tuned = None if args.no_autotune else plan.autotune(iters=3)
    dt_ = plan.dtype
    rng = np.random.default_rng(args.seed + 7)
    bases, params = [], []
    for i, d in enumerate(system.domains):
        bases.append(torch.from_numpy(pair_shapes(d, system.h, system.c)).to("cuda", dt_).contiguous())
        k = len(d.charges)
        p = np.column_stack([rng.uniform(0.5, 5.0, k), np.full(k, 0.05), np.ones(k),
                             [ch.cp[2] - ch.cm[2] if i == 0 else 0.0 for ch in d.charges]])
        params.append(p)
    osc = Oscillators(plan, bases, params)
    src = [torch.empty((4,) + d, dtype=dt_, device="cuda") for d in plan.dims]
    nxt = [torch.empty_like(x) for x in src]
    outs = [torch.empty_like(x) for x in src]
    T_env, w_d = 20.0, 0.8

    def e_ext(l):
        t = l * system.dt
        return math.sin(math.pi * t / T_env) ** 2 * math.sin(w_d * t) if t < T_env else 0.0

    osc.sources(src)
    W, K = args.warmup, args.steps
    if kb > 1:
        W += (-W) % kb          # the timed steps start at a block's first step
    for l in range(W + K + 1):
        if l == W + 1:
            torch.cuda.synchronize()
            plan.lagsum_time()
            plan.profile_lagsum(True)
            t0 = time.perf_counter()
        plan.push_sources(l, src)
        plan.retarded_step(l, outs)
        osc.step(outs, e_ext(l), nxt)
        src, nxt = nxt, src
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.profile_lagsum(False)
    lag_ms, launches = plan.lagsum_time()
    q, qd, phi, psi = osc.state()
    if not (np.all(np.isfinite(q)) and all(bool(torch.isfinite(o).all()) for o in outs)):
        raise RuntimeError("non-finite state")
    n_osc = sum(len(d.charges) for d in system.domains)
    osc_bytes = sum(2 * b.numel() * b.element_size() for b in bases)
    ms_step = 1e3 * el / K
    updates = st["points"] * K / el
    log(f"coupled loop: step {ms_step:.3f} ms ({updates / 1e6:.2f} M updates/s), lag sum {lag_ms / launches:.3f} ms, "
        f"{n_osc} oscillators, shape bytes streamed per step {osc_bytes / 1e9:.2f} GB; "
        f"max |q| domain 0 {np.max(np.abs(q[:16])):.3e}, others {np.max(np.abs(q[16:])):.3e}")
    line = {"metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": {"fp64": "f64"}.get(args.precision, "f32"), "data": "synthetic",
            "config": {"workload": "8 sub-domains of 64^3 points (config 2 geometry), each charge pair a Lorentz "
                                   "oscillator driven by the computed potentials; sources of step l+1 from the "
                                   "potentials of step l on the GPU",
                       "precision": args.precision, "oscillators": n_osc, "lagsum_steps_per_pass": kb,
                       "lagsum_ms": lag_ms / launches, "shape_bytes_per_step": osc_bytes,
                       "max_abs_q": [float(np.max(np.abs(q[:16]))), float(np.max(np.abs(q[16:])))],
                       "autotune": tuned},
            "roofline": {"bound": "hbm", "achieved": round(st["lagsum_bytes"] / (lag_ms / launches * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(st["lagsum_bytes"] / (lag_ms / launches * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": None,
                         "kernel": "k_lagsum" if kb == 1 else f"k_lagsum_block ({kb} steps per pass)",
                         "kernel_ms": round(lag_ms / launches, 4),
                         "algorithmic_bytes_per_launch": st["lagsum_bytes"]},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)
    osc.close()
    plan.close()


def bench_paper(args):
    """The paper's two-molecule geometry with synthetic sources: two
    50 x 50 x 125-point boxes (h = 0.4, dt = 1 as) 90 and 7500 bohr apart,
    each with the history in one spectral ring and split (the far window in
    a ring of its own, fed from a real-space ring in device memory or, at
    7500 bohr, in pinned host memory).  Graph-launched steps."""
    import numpy as np
    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import paper_pair
    K, W = args.steps, args.warmup
    rows = []
    stream = torch.cuda.current_stream()
    for d in (90.0, 7500.0):
        system = paper_pair(d, seed=args.seed)
        last = None
        # a cycle of 64 source steps; warm-up past the deepest lag, so that
        # the timed steps read real history everywhere (and the host tier
        # fetches its snapshots from host memory)
        cyc = 64
        probe = plan_for_system(system, args.precision)
        Wd = max(W, probe.info(1, 0)[1] + 2)
        probe.close()
        srcs = None
        for split, host in ((0, False), (8, False), (8, True)):
            if host and d < 1000:
                continue
            plan = plan_for_system(system, args.precision, stream=stream)
            if split:
                plan.history_split(split)
            if host:
                plan.history_host(True)
            st = plan.stats()
            ws = plan.workspace_bytes
            hb = plan.host_history_bytes
            plan.bind()
            plan.set_green_kernels()
            if srcs is None:
                srcs = make_sources(system, range(cyc), plan.dtype)
            ms, outs = _time_graph(plan, lambda l: srcs[0 if l == 0 else 1 + (l - 1) % (cyc - 1)], Wd, K)
            got = [o.cpu() for o in outs]
            same = None if last is None else all(bool(torch.equal(a, b)) for a, b in zip(last, got))
            if not split:
                last = got
            row = {"d_bohr": d, "split": bool(split), "host_tier": host, "warmup": Wd, "ms_per_step": ms,
                   "updates_per_s": st["points"] * 1e3 / ms, "workspace_gb": ws / 1e9,
                   "host_history_gb": hb / 1e9,
                   "ring_gb": st["ring_bytes"] / 1e9, "real_history_gb": st["history_bytes"] / 1e9,
                   "split_rings": st["split_rings"], "ring_depth": plan.info(0, 0)[3],
                   "cross_window": list(plan.info(1, 0)[:2]), "lagsum_gb": st["lagsum_bytes"] / 1e9}
            if same is not None:
                row["bitwise_equal_to_single_ring"] = same
            log("paper pair " + ", ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}"
                                          for k, v in row.items()))
            rows.append(row)
            plan.close()
            del plan, outs
            torch.cuda.empty_cache()
        del srcs
    best = [r for r in rows if r["d_bohr"] == 7500.0 and r["split"] and not r["host_tier"]][0]
    line = {"metric": METRIC, "value": best["updates_per_s"], "unit": "grid-point updates/s", "n_gpus": 1,
            "steps": K, "warmup": W, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64"}.get(args.precision, "f32"),
            "data": "synthetic",
            "config": {"workload": "the paper's two-molecule geometry: 2 x 50x50x125 points, h=0.4 bohr, "
                                   "dt=1 as, 90 and 7500 bohr apart, single and split history; value: "
                                   "7500 bohr, split",
                       "precision": args.precision, "runs": rows},
            "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def speedup_model(Wp, Lp, dp):
    """The paper's cost ratio for two W x W x L domains side by side in a
    W x d x L box (Sec. III, Eq. of the computational complexity ratio), in
    grid units: retardation steps times N log N per domain pair."""
    diag = math.sqrt(dp * dp + Lp * Lp + Wp * Wp)
    small = Wp * Wp * Lp * math.log(Wp * Wp * Lp)
    big = diag * Wp * dp * Lp * math.log(Wp * dp * Lp)
    inv = (2 * diag * small - 2 * (dp - 2 * Wp) * small + 2 * math.sqrt(2 * Wp * Wp + Lp * Lp) * small) / big
    return 1.0 / inv


def _time_graph(plan, src_at, W, K):
    """ms per graph-launched step after W warm-up steps (the sources for
    step l come from src_at(l), copied into the captured buffers)."""
    import torch
    outs = [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    buf = [torch.empty_like(o) for o in outs]
    plan.push_sources(0, src_at(0))
    plan.retarded_step(0, outs)
    plan.capture_step(buf, outs)
    for l in range(1, W + K + 1):
        if l == W + 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        torch._foreach_copy_(buf, src_at(l))
        plan.launch_step(l)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / K, outs


def bench_sweep(args):
    """Measured form of the paper's single- vs multi-domain cost comparison
    (Sec. III, Fig. 3): two W x W x L domains side by side, the box that
    encloses both W x d x L.  Per d: the step time of the two-domain plan and
    of the one-domain plan (same sources, zero between the domains), the
    agreement of the two on the sub-domain points, and the model's ratio."""
    import numpy as np
    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import enclosing_domain, wire_pair
    Wp, Lp = 32, 128
    both = [72, 96, 128, 160, 192, 224, 256]
    multi_only = [512, 1024, 2048, 4096]
    precision = args.precision
    K = args.steps
    rows = []
    stream = torch.cuda.current_stream()
    for dp in both + multi_only:
        system = wire_pair(W=Wp, L=Lp, d=dp, n_pairs=8, seed=args.seed)
        row = {"d_points": dp, "d_over_L": dp / Lp, "d_bohr": round(dp * system.h, 2),
               "speedup_model": speedup_model(Wp, Lp, dp)}
        plan = plan_for_system(system, precision, stream=stream)
        depth = max(plan.info(0, n)[3] for n in range(2))
        row["multi_lagsum_bytes"] = plan.stats()["lagsum_bytes"]
        row["multi_ring_depth"] = depth
        plan.bind()
        plan.set_green_kernels()
        W = depth + 2
        src = make_sources(system, range(W + K + 1), plan.dtype)
        row["ms_multi"], outs_m = _time_graph(plan, lambda l: src[l], W, K)
        if dp in both:
            encl, blocks = enclosing_domain(system)
            dims = tuple(encl.domains[0].dims)
            big_src = []
            for l in range(W + K + 1):
                big = torch.zeros((4,) + dims, dtype=plan.dtype, device="cuda")
                for n, b in enumerate(blocks):
                    big[(slice(None),) + b] = src[l][n]
                big_src.append([big])
            sp = plan_for_system(encl, precision, stream=stream)
            row["single_lagsum_bytes"] = sp.stats()["lagsum_bytes"]
            sdepth = sp.info(0, 0)[3]
            sp.bind()
            sp.set_green_kernels()
            # the same number of steps, so both end on the same step
            row["ms_single"], outs_s = _time_graph(sp, lambda l: big_src[l], W, K)
            big = outs_s[0].double()
            diff = 0.0
            for n, b in enumerate(blocks):
                cut = big[(slice(None),) + b]
                ref = outs_m[n].double()
                diff = max(diff, float(torch.max(torch.abs(cut - ref)) / torch.max(torch.abs(ref))))
            row["rel_diff_single_vs_multi"] = diff
            row["speedup_measured"] = row["ms_single"] / row["ms_multi"]
            row["single_ring_depth"] = sdepth
            sp.close()
            del sp, outs_s, big_src
        plan.close()
        del plan, outs_m, src
        torch.cuda.empty_cache()
        log("sweep " + ", ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}" for k, v in row.items()))
        rows.append(row)
    last = [r for r in rows if "speedup_measured" in r][-1]
    ms_m = [r["ms_multi"] for r in rows]
    line = {"metric": "multi-domain speedup over one enclosing domain (measured step time ratio)",
            "value": last["speedup_measured"], "unit": "x", "n_gpus": 1, "steps": K, "warmup": "ring depth + 2",
            "ms_per_step": last["ms_multi"], "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": {"fp64": "f64"}.get(precision, "f32"), "data": "synthetic",
            "config": {"workload": f"two {Wp}x{Wp}x{Lp}-point domains side by side along y, h=0.3 bohr, dt=0.01; "
                                   f"enclosing box {Wp}x d x {Lp}; value at d={last['d_points']} points",
                       "precision": precision,
                       "multi_ms_spread_over_d": [min(ms_m), max(ms_m)],
                       "sweep": rows},
            "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_mlp(args):
    """The far-pair surrogate network at its config-5 shape (8450 inputs,
    2 x 256 tanh hidden, 80 outputs, linear skip): Adam training steps at a
    minibatch of 2048 and inference over 990 far pairs, on random inputs and
    the training run's initial weights.  Every product runs in the library's
    FP32 matrix-core kernel; the roofline is the products' FP32 flops over the
    whole timed step (its other kernels included) against the FP32 MFMA peak."""
    import numpy as np
    import torch
    from paper_2311_15429_amd.mlp import Mlp
    ni, H, no, B, Bi = 8450, 256, 80, 2048, 990
    W, K = max(args.warmup, 3), args.steps
    stream = torch.cuda.current_stream()
    mlp = Mlp(ni, H, no, B, stream=stream)
    g = torch.Generator(device="cpu").manual_seed(args.seed)
    parts = [torch.randn(ni * H, generator=g) / math.sqrt(ni), torch.zeros(H),
             torch.randn(H * H, generator=g) / math.sqrt(H), torch.zeros(H),
             torch.randn(H * no, generator=g) / math.sqrt(H), torch.zeros(no),
             torch.randn(ni * no, generator=g) / math.sqrt(ni)]
    mlp.set_params(torch.cat(parts).float())
    x = torch.randn((B, ni), generator=g).float().cuda()
    t = torch.randn((B, no), generator=g).float().cuda()
    xi = x[:Bi].contiguous()
    y = torch.empty((Bi, no), dtype=torch.float32, device="cuda")

    def timed(fn, n_warm, n):
        for _ in range(n_warm):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    ms_train = timed(lambda: mlp.train_step(x, t, 1e-4), W, K)
    ms_infer = timed(lambda: mlp.forward(xi, out=y), W, K)
    fl_train = 2.0 * B * (2 * ni * H + 3 * H * H + 3 * H * no + 2 * ni * no)
    fl_infer = 2.0 * Bi * (ni * H + H * H + H * no + ni * no)
    peak = 157.3
    ach = fl_train / (ms_train * 1e-3) / 1e12
    log(f"mlp: train step (batch {B}) {ms_train:.3f} ms = {ach:.1f} TFLOP/s; "
        f"inference ({Bi} pairs) {ms_infer:.3f} ms = {fl_infer / (ms_infer * 1e-3) / 1e12:.1f} TFLOP/s")
    line = {"metric": "surrogate network training samples/s (Adam steps on the GPU)",
            "value": B / (ms_train * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": ms_train, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"far-pair network {ni} -> {H} -> {H} -> {no} (tanh, linear skip), "
                                   f"minibatch {B}; inference over {Bi} far pairs",
                       "train_gflop_per_step": fl_train / 1e9, "infer_ms": ms_infer,
                       "infer_gflop": fl_infer / 1e9,
                       "infer_tflops": fl_infer / (ms_infer * 1e-3) / 1e12},
            "roofline": {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(ach / peak, 4), "traffic": None,
                         "kernel": "k_gemm (FP32 matrix cores); achieved over the whole step, its split-K "
                                   "reductions, loss, tanh, column-sum and Adam kernels included"},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=96, help="timed steps (96: whole blocks of 8 lag-sum steps)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default=None, choices=["fp32", "fp32_ring_fp16", "fp32_ring_bf16", "fp32_ring_i16", "fp64"],
                    help="default: fp32 (scale, batched, small: fp64 always, sweep, coupled, paper); "
                         "fp32_ring_i16 for the surrogate workload, fp32_ring_fp16 for batched_scaled")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fill", action="store_true",
                    help="scale workload: time from step 1 on instead of after the history fill")
    ap.add_argument("--lagsum-unroll", type=int, default=None, choices=[1, 2, 4])
    ap.add_argument("--lagsum-steps", type=int, default=8, choices=[1, 2, 4, 8, 16],
                    help="scale and surrogate workloads: steps of the lag sum per pass over the history (1: "
                         "every step reads the whole history)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default lag-sum schedule")
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "batched", "batched_scaled", "surrogate", "small", "sweep", "coupled", "paper", "mlp"],
                    help="scale: 8 x 64^3 (the metric's workload); batched: 64 independent systems "
                         "(2-16 domains of 32^3-96^3) in waves of target groups; batched_scaled: the batched "
                         "recipe at 16^3-32^3 and 2-8 domains in one plan, one graph launch per step; "
                         "surrogate: 32 x 48^3 in a 2000-bohr box with the learned far-pair surrogate; "
                         "small: 2 x 16^3 in FP64 beside the oracle's full run; "
                         "sweep: two 32x32x128 domains vs the box enclosing both, over the distance; "
                         "coupled: config 2 with oscillator sources driven by the potentials; "
                         "paper: the paper's two-molecule geometry, single and split history; "
                         "mlp: the surrogate network's training and inference at its config-5 shape")
    ap.add_argument("--far", default="learned", choices=["learned", "multipole", "hybrid"],
                    help="surrogate workload: far-pair terms from the trained network, the analytic "
                         "multipole, or the multipole plus a network trained on its residual")
    ap.add_argument("--teacher-seeds", type=int, nargs="+", default=[101, 102, 103])
    ap.add_argument("--teacher-audit", type=int, default=3, help="audit sources per teacher system")
    ap.add_argument("--audit", type=int, nargs="*", default=[0, 1], help="audit sources of the timed run")
    ap.add_argument("--readmit", type=float, default=0.5,
                    help="surrogate workload: re-admission factor of fallen-back pairs (0: never)")
    ap.add_argument("--oracle-targets", type=int, default=3)
    ap.add_argument("--oracle-points", type=int, default=24)
    ap.add_argument("--wave-steps", type=int, default=8,
                    help="batched: timed graph replays per wave (default one block of 8 lag-sum steps)")
    ap.add_argument("--wave-warmup", type=int, default=1, help="batched: warm-up replays per wave")
    ap.add_argument("--wave-gb", type=float, default=0.0,
                    help="batched workload: cap of a wave's workspace in GB (default: the free device memory)")
    ap.add_argument("--no-plain-baseline", dest="plain_baseline", action="store_false",
                    help="surrogate workload: skip the measured plain FP32 run (waves of target groups)")
    ap.add_argument("--split-gap", type=int, default=8,
                    help="batched workload: history split gap of the wave plans (lags)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.precision is None and args.workload not in ("batched", "batched_scaled", "surrogate"):
        args.precision = "fp32"

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU path (sharding by source "
              "domain with one reduce-scatter per step) is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import config2

    if args.workload == "mlp":
        return bench_mlp(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "batched_scaled":
        return bench_batched_scaled(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "coupled":
        return bench_coupled(args)
    if args.workload == "paper":
        return bench_paper(args)
    system = config2(args.seed)
    workload = "8 sub-domains of 64^3 points, h=0.3 bohr, 400-bohr box, dt=0.01, FFT pad 128^3"
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, args.precision, stream=stream)
    if args.lagsum_steps > 1:
        plan.set_tuning("lagsum_steps", args.lagsum_steps)
    st = plan.stats()
    log(f"plan: triples/step {st['n_triples']}, spectra {st['n_spectra']}, ring reads/step {st['n_entries']}, "
        f"workspace {plan.workspace_bytes / 1e9:.1f} GB, lag-sum bytes/launch {st['lagsum_bytes'] / 1e9:.2f} GB")
    t0 = time.perf_counter()
    plan.bind()
    plan.set_green_kernels()
    torch.cuda.synchronize()
    t_green = time.perf_counter() - t0
    log(f"bind + Green spectra: {t_green:.2f} s")
    tuned = None
    if args.lagsum_unroll:
        plan.set_tuning("lagsum_unroll", args.lagsum_unroll)
    elif not args.no_autotune:
        tuned = plan.autotune(iters=3)
        log(f"autotune: {tuned}")

    W, K = args.warmup, args.steps
    dtype = plan.dtype
    # fill the history: run every step up to the deepest ring slot first, so
    # that the timed steps read real history in every (target, source, lag)
    # triple (the kernel's bytes and schedule do not depend on it)
    F = 0 if args.no_fill else max(plan.info(n, n)[3] for n in range(plan.n_dom))
    kb = plan.get_tuning("lagsum_steps")
    # with kb steps per pass the timed steps start at a block's first step, so
    # every pass that serves a timed step is timed (with K not a multiple of
    # kb the last pass also serves steps after the timed region: the figure
    # then errs on the slow side)
    if kb > 1:
        F += (-(F + W)) % kb
    gen = SourceGen(system, dtype)
    outs = [torch.empty((4,) + d, dtype=dtype, device="cuda") for d in plan.dims]
    t0 = time.perf_counter()
    for l in range(0, F + 1):
        plan.push_sources(l, gen(l))
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    log(f"history fill: steps 0..{F} in {time.perf_counter() - t0:.1f} s")
    src = [gen(l) for l in range(F + 1, F + W + K + 1)]
    torch.cuda.synchronize()

    for l in range(F + 1, F + W + 1):
        plan.push_sources(l, src[l - F - 1])
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    plan.lagsum_time()
    plan.profile_lagsum(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(F + W + 1, F + W + K + 1):
        plan.push_sources(l, src[l - F - 1])
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = F + W + K
    plan.profile_lagsum(False)
    lag_ms, launches = plan.lagsum_time()
    assert launches == (K if kb == 1 else sum(1 for l in range(F + W + 1, F + W + K + 1) if (l - 1) % kb == 0))
    if not all(bool(torch.isfinite(o).all()) for o in outs):
        raise RuntimeError("non-finite output")

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del a, b

    ms_step = 1e3 * el / K
    updates = st["points"] * K / el
    lag_avg_s = lag_ms / launches / 1e3
    achieved = st["lagsum_bytes"] / lag_avg_s / 1e9
    traffic = traffic_from_profiles("config2" if kb == 1 else f"config2_blocked{kb}", args.precision)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_lagsum", "kernel_ms": round(lag_avg_s * 1e3, 4),
            "algorithmic_bytes_per_launch": st["lagsum_bytes"]}
    if kb > 1:
        roof["kernel"] = f"k_lagsum_block ({kb} steps per pass)"
        roof["lagsum_bytes_per_step"] = st["lagsum_bytes"] / kb
    log(f"step {ms_step:.3f} ms, lag-sum {lag_avg_s * 1e3:.3f} ms ({achieved:.0f} GB/s), "
        f"{updates / 1e6:.2f} M updates/s")
    # the practical read bandwidth of this device (a plain read stream of 4
    # GiB through the library's calibration kernel), beside the lag sum
    from paper_2311_15429_amd.calib import read_stream_gbs
    rs, rs_cfg = read_stream_gbs()
    roof["read_stream_gbs"] = round(rs, 1)
    roof["read_stream_launch"] = {"unroll": rs_cfg[0], "blocks_per_cu": rs_cfg[1]}
    roof["frac_of_read_stream"] = round(achieved / rs, 4)
    log(f"read stream: {rs:.0f} GB/s ({rs / HBM_PEAK_GBS:.1%} of peak, unroll {rs_cfg[0]}, "
        f"{rs_cfg[1]} blocks per CU); the lag sum runs at {achieved / rs:.1%} of it")

    cpu, err = None, None
    if not args.no_cpu_baseline:
        del src
        torch.cuda.empty_cache()
        log(f"cpu baseline (oracle) at step {last} ...")

        def gpu_values(s, idx):
            sel = torch.from_numpy(np.asarray(idx, dtype=np.int64)).to("cuda")
            return outs[s].reshape(4, -1)[:, sel].double().cpu().numpy()

        cpu, err = cpu_baseline(system, args.cpu_seconds, last, gpu_values)
        log(f"cpu baseline: {cpu['value']:.1f} updates/s on {cpu['cores']} cores")
        log(f"rel err vs FP64 oracle at step {last} ({err['points']} points): max "
            + " ".join(f"{v:.2e}" for v in err["max"]) + ", rms " + " ".join(f"{v:.2e}" for v in err["rms"]))

    dtype_name = {"fp64": "f64"}.get(args.precision, "f32")
    line = {
        "metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": workload, "precision": args.precision, "sub_domains": 8, "grid": [64, 64, 64],
                   "h_bohr": 0.3, "dt_au": 0.01, "c_au": 137.036, "seed": args.seed,
                   "triples_per_step": st["n_triples"], "ring_reads_per_step": st["n_entries"],
                   "history_fill_steps": F, "timed_steps": [F + W + 1, last],
                   "lagsum_passes_timed": launches,
                   "green_setup_s": round(t_green, 3),
                   "lagsum_steps_per_pass": kb,
                   "lagsum_unroll": plan.get_tuning("lagsum_unroll"),
                   "lagsum_persistent": plan.get_tuning("lagsum_persistent"),
                   "fft_lds": plan.get_tuning("fft_lds"),
                   "autotuned": tuned is not None},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_err_vs_fp64_sampled": err,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
