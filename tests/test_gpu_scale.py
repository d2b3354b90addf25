"""Parity at the benchmark's full size, in its launch configuration, after the
history has filled, and the reduced-precision history rings against the FP64
oracle.

Full size: 8 sub-domains of 64^3 points (FFT pad 128^3, history rings of
234-381 spectra, cross-pair windows from lag 42 to lag 380), FP32, sources
generated per step on the GPU from the same seeded factors the oracle
evaluates in FP64.  The oracle computes sampled target points one by one (each
is a direct sum over all 2,097,152 source points).  The sampled steps include
the first arrival of the nearest (lag 42) and the farthest (lag 340) cross
pair and steps past the deepest lag (380), where every (target, source, lag)
triple of the lag sum reads real history, including the deepest ring slots
and their wrap-around.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import GpuSourceGen, cpu_sample_fn, log, pick_points
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# oracle values shared by the tests of this module: {(system name, s, l): [n_pts][4]}
_ORACLE = {}


def _windows(system, precision="fp32"):
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, precision)
    n = len(system.domains)
    lo = np.array([[p.info(s, m)[0] for m in range(n)] for s in range(n)])
    hi = np.array([[p.info(s, m)[1] for m in range(n)] for s in range(n)])
    p.close()
    return lo, hi


def _picks(system, n_pts, seed):
    rng = np.random.default_rng(seed)
    return {s: pick_points(d.dims, n_pts, rng) for s, d in enumerate(system.domains)}


def _run_sampled(system, precision, steps_out, picks, tune=None):
    from paper_2311_15429_amd import plan_for_system
    stream = torch.cuda.current_stream()
    plan = plan_for_system(system, precision, stream=stream)
    for k, v in (tune or {}).items():
        plan.set_tuning(k, v)
    plan.bind()
    plan.set_green_kernels()
    gen = GpuSourceGen(system, plan.dtype)
    outs = [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    sel = [torch.from_numpy(picks[s]).to("cuda") for s in range(len(system.domains))]
    got = {}
    for l in range(max(steps_out) + 1):
        plan.push_sources(l, gen.step(l))
        plan.retarded_step(l, outs)
        if l in steps_out:
            got[l] = [o.reshape(4, -1)[:, sel[s]].double().cpu().numpy() for s, o in enumerate(outs)]
            log(f"  step {l} collected")
    torch.cuda.synchronize()
    plan.close()
    return got


def _oracle_values(system, picks, l, fn):
    out = []
    for s in range(len(system.domains)):
        key = (system.name, s, l, picks[s].tobytes())
        if key not in _ORACLE:
            _ORACLE[key] = oracle.potential_points(system, s, picks[s], l, fn)
        out.append(_ORACLE[key].T)
    return out


def _compare(system, got, picks, steps_out, label):
    """Per step and component: max and RMS of |gpu - oracle| over the sampled
    points of every domain, divided by max |oracle| (the error definition of
    every parity bar)."""
    fn = cpu_sample_fn(system)
    errs = {}
    for l in steps_out:
        ref = _oracle_values(system, picks, l, fn)
        g = np.concatenate(got[l], axis=1)
        r = np.concatenate(ref, axis=1)
        scale = np.max(np.abs(r), axis=1)
        e_max = np.max(np.abs(g - r), axis=1) / scale
        e_rms = np.sqrt(np.mean((g - r) ** 2, axis=1)) / scale
        errs[l] = (e_max, e_rms)
        fmt = lambda v: "[" + " ".join(f"{x:.2e}" for x in v) + "]"   # noqa: E731
        log(f"  [{label}] step {l}: max rel err (v Ax Ay Az) {fmt(e_max)}, rms {fmt(e_rms)}")
    return errs


def _active_triples(lo, hi, l):
    """(target, source, lag) triples whose ring slot holds history at step l."""
    n = lo.shape[0]
    return int(sum(max(0, min(hi[s, m], l - 1) - lo[s, m] + 1) for s in range(n) for m in range(n)))


@pytest.mark.timeout(900)
def test_config2_full_size_steady_state_fp32():
    """Config 2 in FP32 past the deepest lag: 128 points per domain (corners,
    face centres, edge midpoints, face and interior points) at 8 steps, from
    the first step through the nearest and farthest first arrivals to two
    steps past the deepest lag, within 2e-5 of the FP64 oracle."""
    system = sy.config2(0)
    lo, hi = _windows(system)
    off = ~np.eye(8, dtype=bool)
    near, far, deep = int(lo[off].min()), int(lo[off].max()), int(hi.max())
    assert (near, far, deep) == (42, 340, 380)
    steps_out = [1, near + 1, 120, 230, far + 1, 360, deep + 2, deep + 21]
    total = _active_triples(lo, hi, 10 ** 9)
    for l in steps_out:
        log(f"  step {l}: {_active_triples(lo, hi, l)} of {total} triples hold history")
    assert _active_triples(lo, hi, deep + 2) == total
    picks = _picks(system, 128, seed=0)
    log("config2 full size: GPU run")
    got = _run_sampled(system, "fp32", steps_out, picks)
    log("config2 full size: oracle")
    errs = _compare(system, got, picks, steps_out, "fp32")
    for l, (e_max, _) in errs.items():
        assert np.all(e_max <= 2e-5), (l, e_max)


# 16-bit history rings at the full shape: the block-floating-point I16 ring
# meets the 1e-4 mixed-precision bar; the FP16 ring (11 significant bits)
# does not (2.1e-4 measured past the deepest lag), its bar states what it reaches
FULL_16BIT_BARS = {"fp32_ring_i16": 1e-4, "fp32_ring_fp16": 3e-4}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32_ring_i16", "fp32_ring_fp16"])
def test_config2_full_size_16bit_ring(precision):
    """Config 2 with the history ring in 16 bits (FP32 FFTs and accumulation)
    at the full shape, up to past the deepest lag, against the FP64 oracle at
    32 points per domain."""
    system = sy.config2(0)
    steps_out = [230, 382, 401]
    picks = _picks(system, 32, seed=5)
    log(f"config2 full size, {precision}: GPU run")
    got = _run_sampled(system, precision, steps_out, picks)
    errs = _compare(system, got, picks, steps_out, precision)
    for l, (e_max, _) in errs.items():
        assert np.all(e_max <= FULL_16BIT_BARS[precision]), (l, e_max)


@pytest.mark.parametrize("unroll", [1, 4])
def test_lagsum_unroll_variants_agree(unroll):
    """Every lag-sum schedule gives the same result as the default up to
    rounding order (small uneven system, FP32)."""
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


# measured worst errors (max over steps 1..450 and components) of the 32^3 twin
# stay below these bars.  The I16 ring meets the 1e-4 mixed-precision target;
# the FP16 ring (11 significant bits) misses it once the windows fill (1.25e-4
# at step 450) and the BF16 ring (8 bits) misses it by 10x (1.0e-3)
TWIN_BARS = {"fp32": 2e-5, "fp32_ring_i16": 1e-4, "fp32_ring_fp16": 2e-4, "fp32_ring_bf16": 2e-3}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp32_ring_i16", "fp32_ring_fp16", "fp32_ring_bf16"])
def test_twin_reduced_precision_rings(precision):
    """Config-2 centres and sources resampled at 32^3 (h = 0.6): FP32 FFTs and
    accumulation with the history ring in FP32, scaled FP16 or BF16, against the
    FP64 oracle at 128 sampled points per domain, every 50th step through 450
    plus the nearest and farthest first arrivals."""
    twin = sy.config3_twin(sy.config2(0), 32)
    lo, hi = _windows(twin)
    off = ~np.eye(8, dtype=bool)
    near, far = int(lo[off].min()), int(lo[off].max())
    steps_out = sorted(set([1, near + 1, far + 1] + list(range(50, 451, 50))))
    picks = _picks(twin, 128, seed=1)
    log(f"twin {precision}: GPU run, steps {steps_out}")
    got = _run_sampled(twin, precision, steps_out, picks)
    errs = _compare(twin, got, picks, steps_out, precision)
    worst = np.max([e[0] for e in errs.values()], axis=0)
    worst_rms = np.max([e[1] for e in errs.values()], axis=0)
    log(f"  [{precision}] worst over steps: max " + " ".join(f"{x:.2e}" for x in worst)
        + ", rms " + " ".join(f"{x:.2e}" for x in worst_rms))
    assert np.all(worst <= TWIN_BARS[precision]), worst
