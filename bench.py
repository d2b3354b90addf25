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
import hashlib
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


def kernel_source_sha():
    h = hashlib.sha1()
    for f in ("lagsum.hip", "rpot_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2311_15429_amd", "csrc", f), "rb").read())
    return h.hexdigest()


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
    if not ent or ent.get("kernel_source_sha") != kernel_source_sha():
        return None
    return ent.get("traffic_bytes_per_launch")


def cpu_baseline(system, target_seconds):
    """The oracle (FP64 direct sum) on a bounded sample of the same workload:
    grid points of target domain 0 at one step, all 8 source domains."""
    import numpy as np
    import oracle
    from synth.sources import spatial_factors, time_factors
    l = 200
    t = l * system.dt
    dom0 = system.domains[0]
    cache = {}
    for n, d in enumerate(system.domains):
        rmin, rmax = oracle.box_distance_range(dom0, d, system.h)
        j0, j1 = oracle.needed_sample_range(t, rmin, rmax, system.dt, system.c, self_cell=(n == 0))
        B = spatial_factors(d, system.h, system.c)
        nt = B.shape[0]
        js = np.arange(j0, j1 + 1)
        A = time_factors(d, system.dt, np.concatenate([[0], js]))
        S = (A @ B.reshape(nt, -1)).reshape(len(js) + 1, 4, -1)
        cache[n] = (j0, S)

    def fn(n, a, b):
        j0, S = cache[n]
        if a == 0 and b == 0:
            return S[:1]
        return S[1 + a - j0: 2 + b - j0]

    rng = np.random.default_rng(0)
    c1 = oracle.self_cell_c1()
    npts = 8
    while True:
        idx = np.sort(rng.choice(dom0.n_points, size=npts, replace=False))
        t0 = time.perf_counter()
        oracle.potential_points(system, 0, idx, l, fn, c1=c1)
        el = time.perf_counter() - t0
        if el >= 0.5 * target_seconds or npts >= dom0.n_points:
            break
        npts = min(dom0.n_points, int(npts * min(64.0, max(2.0, target_seconds / max(el, 1e-3)))))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": npts / el, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{npts} grid points of domain 0 (all 8 source domains, 2,097,152 source points each "
                      f"update) at step {l}; {el:.1f} s of oracle time",
            "seconds": el}


def bench_batched(args):
    """64 independent systems with uneven domain counts and grid sizes in one
    plan; each step is one replay of the captured graph."""
    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import config4
    system = config4(args.seed, sizes=(16, 24, 32), n_dom_range=(2, 8))
    precision = args.precision if args.precision != "fp32" else "fp32_ring_fp16"
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
    src = make_sources(system, range(W + K + 1), plan.dtype)
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
    line = {"metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 independent systems, 2-8 sub-domains each of 16^3/24^3/32^3 points, "
                                   "h=0.3 bohr, separations 20-300 bohr, dt=0.01, one graph launch per step",
                       "precision": precision, "domains": len(system.domains),
                       "triples_per_step": st["n_triples"], "lagsum_bytes": st["lagsum_bytes"],
                       "workspace_bytes": plan.workspace_bytes, "autotune": tuned}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_ring_fp16", "fp32_ring_bf16", "fp64"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lagsum-unroll", type=int, default=None, choices=[1, 2, 4])
    ap.add_argument("--no-autotune", action="store_true", help="keep the default lag-sum schedule")
    ap.add_argument("--workload", default="scale", choices=["scale", "batched"],
                    help="scale: 8 x 64^3 (the metric's workload); batched: 64 independent systems "
                         "(2-8 domains of 16^3/24^3/32^3) in one plan, one graph launch per step")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU path (sharding by source "
              "domain with one reduce-scatter per step) is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_15429_amd import plan_for_system
    from synth.sources import config2, config4

    if args.workload == "batched":
        return bench_batched(args)
    system = config2(args.seed)
    workload = "8 sub-domains of 64^3 points, h=0.3 bohr, 400-bohr box, dt=0.01, FFT pad 128^3"
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, args.precision, stream=stream)
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
    src = make_sources(system, range(W + K + 1), dtype)
    outs = [torch.empty((4,) + d, dtype=dtype, device="cuda") for d in plan.dims]
    torch.cuda.synchronize()

    plan.push_sources(0, src[0])
    plan.retarded_step(0, outs)
    for l in range(1, W + 1):
        plan.push_sources(l, src[l])
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    plan.lagsum_time()
    plan.profile_lagsum(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(W + 1, W + K + 1):
        plan.push_sources(l, src[l])
        plan.retarded_step(l, outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.profile_lagsum(False)
    lag_ms, launches = plan.lagsum_time()
    assert launches == K
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
    traffic = traffic_from_profiles("config2", args.precision)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_lagsum", "kernel_ms": round(lag_avg_s * 1e3, 4),
            "algorithmic_bytes_per_launch": st["lagsum_bytes"]}
    log(f"step {ms_step:.3f} ms, lag-sum {lag_avg_s * 1e3:.3f} ms ({achieved:.0f} GB/s), "
        f"{updates / 1e6:.2f} M updates/s")

    cpu = None
    if not args.no_cpu_baseline:
        del src
        torch.cuda.empty_cache()
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(system, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.1f} updates/s on {cpu['cores']} cores")

    dtype_name = {"fp64": "f64"}.get(args.precision, "f32")
    line = {
        "metric": METRIC, "value": updates, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": workload, "precision": args.precision, "sub_domains": 8, "grid": [64, 64, 64],
                   "h_bohr": 0.3, "dt_au": 0.01, "c_au": 137.036, "seed": args.seed,
                   "triples_per_step": st["n_triples"], "ring_reads_per_step": st["n_entries"],
                   "green_setup_s": round(t_green, 3),
                   "lagsum_unroll": plan.get_tuning("lagsum_unroll"),
                   "lagsum_persistent": plan.get_tuning("lagsum_persistent"),
                   "autotuned": tuned is not None},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
