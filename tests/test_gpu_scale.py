"""Parity at the benchmark's full size and in its launch configuration, and the
reduced-precision history rings against the FP64 oracle.

Full size: 8 sub-domains of 64^3 points (FFT pad 128^3, history rings of
211-381 spectra), FP32, sources generated per step on the GPU from the same
seeded factors the oracle evaluates in FP64.  The oracle computes sampled target
points one by one (each is a direct sum over all 2,097,152 source points).
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import GpuSourceGen, cpu_sample_fn, log
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run_sampled(system, precision, steps_out, n_pts, seed=0, unroll=None, tune=None):
    from paper_2311_15429_amd import plan_for_system
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, precision, stream=stream)
    if unroll is not None:
        plan.set_tuning("lagsum_unroll", unroll)
    for k, v in (tune or {}).items():
        plan.set_tuning(k, v)
    plan.bind()
    plan.set_green_kernels()
    gen = GpuSourceGen(system, plan.dtype)
    outs = [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    rng = np.random.default_rng(seed)
    picks = {}
    for s, d in enumerate(system.domains):
        idx = rng.choice(d.n_points, size=n_pts - 2, replace=False)
        picks[s] = np.unique(np.concatenate([idx, [0, d.n_points - 1]]))
    got = {}
    for l in range(max(steps_out) + 1):
        plan.push_sources(l, gen.step(l))
        plan.retarded_step(l, outs)
        if l in steps_out:
            got[l] = [o.double().cpu().numpy().reshape(4, -1)[:, picks[s]] for s, o in enumerate(outs)]
            log(f"  step {l} collected")
    torch.cuda.synchronize()
    plan.close()
    return got, picks


def _compare(system, got, picks, steps_out, fn, label):
    errs = {}
    for l in steps_out:
        g_all, r_all = [], []
        for s in range(len(system.domains)):
            ref = oracle.potential_points(system, s, picks[s], l, fn)
            g_all.append(got[l][s])
            r_all.append(ref.T)
        g = np.concatenate(g_all, axis=1)
        r = np.concatenate(r_all, axis=1)
        e_max = np.max(np.abs(g - r), axis=1) / np.max(np.abs(r), axis=1)
        e_rms = np.sqrt(np.mean((g - r) ** 2, axis=1)) / np.max(np.abs(r), axis=1)
        errs[l] = (e_max, e_rms)
        log(f"  [{label}] step {l}: max rel err {np.array2string(e_max, precision=2)}, "
            f"rms {np.array2string(e_rms, precision=2)}")
    return errs


def test_config2_full_size_sampled_fp32():
    system = sy.config2(0)
    steps_out = [1, 45, 110]
    log("config2 full size: GPU run")
    got, picks = _run_sampled(system, "fp32", steps_out, n_pts=16)
    # retardation is exercised: some cross pairs have lags inside the run
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, "fp32")
    lo = min(p.info(s, n)[0] for s in range(8) for n in range(8) if s != n)
    assert lo < 110
    log("config2 full size: oracle")
    errs = _compare(system, got, picks, steps_out, cpu_sample_fn(system), "fp32")
    for l, (e_max, _) in errs.items():
        assert np.all(e_max <= 2e-5), (l, e_max)


@pytest.mark.parametrize("unroll", [1, 4])
def test_lagsum_unroll_variants_agree(unroll):
    """Every lag-sum schedule gives the same result as the default up to
    rounding order (small uneven system, FP32)."""
    from gpu_helpers import run_gpu
    from test_gpu_parity import _uneven_system
    s = _uneven_system(8)
    S = sy.sample_sources(s, range(13))
    ref = oracle.potential_full(s, S, [12])[0]
    from paper_2311_15429_amd import plan_for_system
    stream = torch.cuda.current_stream()
    plan = plan_for_system(s, "fp32", stream=stream)
    plan.set_tuning("lagsum_unroll", unroll)
    assert plan.get_tuning("lagsum_unroll") == unroll
    plan.bind()
    plan.set_green_kernels()
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in plan.dims]
    for l in range(13):
        plan.push_sources(l, [torch.from_numpy(S[n][l].reshape((4,) + plan.dims[n])).float().cuda()
                              for n in range(3)])
        plan.retarded_step(l, outs)
    g = np.concatenate([o.double().cpu().numpy().reshape(4, -1) for o in outs], axis=1)
    r = np.concatenate(ref, axis=1)
    assert np.all(np.max(np.abs(g - r), axis=1) / np.max(np.abs(r), axis=1) <= 2e-5)


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("fp32_ring_fp16", 2e-4), ("fp32_ring_bf16", 2e-3)])
def test_twin_reduced_precision_rings(precision, tol):
    """Config-2 centres and sources resampled at 32^3 (h = 0.6): FP32 FFTs and
    accumulation with the history ring in FP32, scaled FP16 or BF16, against the
    FP64 oracle at sampled points."""
    twin = sy.config3_twin(sy.config2(0), 32)
    steps_out = [1, 60, 130]
    log(f"twin {precision}: GPU run")
    got, picks = _run_sampled(twin, precision, steps_out, n_pts=48, seed=1)
    errs = _compare(twin, got, picks, steps_out, cpu_sample_fn(twin), precision)
    worst = max(float(e[0].max()) for e in errs.values())
    log(f"  [{precision}] worst max rel err {worst:.3e}")
    assert worst <= tol
