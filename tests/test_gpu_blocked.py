"""Blocked lag-sum steps (RP_TUNE_LAGSUM_STEPS): kb steps share one pass over
the history, and each step adds its own lags m < i once its sources are in.
Every step must still equal the FP64 oracle's potential of that step: at
every step of small systems (each phase of several blocks), through captured
graphs interleaved with eager steps, and at the full config-2 shape past the
deepest lag."""
import numpy as np
import pytest

import oracle
from gpu_helpers import GpuSourceGen, log, pick_points, rel_err, run_gpu
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision,kb,tol", [("fp32", 2, 2e-5), ("fp32", 4, 2e-5), ("fp32", 8, 2e-5),
                                               ("fp32", 16, 2e-5), ("fp32_ring_i16", 8, 1e-4),
                                               ("fp32_ring_i16", 16, 1e-4)])
def test_blocked_steps_match_the_oracle_at_every_step(precision, kb, tol):
    from test_gpu_parity import _uneven_system
    s = _uneven_system(8)
    L = 3 * kb + 5                       # several blocks and a partial one
    S = sy.sample_sources(s, range(L + 1))
    got = run_gpu(s, precision, S, tune={"lagsum_steps": kb})
    plain = run_gpu(s, precision, S)
    ref = oracle.potential_full(s, S, range(L + 1))
    worst, worst_d = 0.0, 0.0
    for l in range(L + 1):
        e = rel_err(got[l], ref[l])
        d = rel_err(got[l], plain[l])
        worst, worst_d = max(worst, float(e.max())), max(worst_d, float(d.max()))
        assert np.all(e <= tol), (l, e)
    log(f"{precision}, {kb} steps per pass, {L + 1} steps: vs oracle {worst:.2e}, vs unblocked {worst_d:.2e}")


def _spread_system(seed=3):
    """Three uneven domains far enough apart (cross-pair windows from lag 9 on)
    that a blocked step's own lags m < 8 are the self pairs' alone, with x
    pads of 48 and 96 (x-lines that cross the 256-frequency tiles)."""
    rng = np.random.default_rng(seed)
    h = 0.5
    doms = [sy.Domain((20, 9, 20), np.array([0.0, 0.0, 0.0])),
            sy.Domain((40, 8, 26), np.array([36.0, 3.0, -2.0])),
            sy.Domain((12, 6, 14), np.array([-3.0, 34.0, 8.0]))]
    for d in doms:
        lo = d.origin
        hi = d.origin + h * (np.array(d.dims) - 1)
        for _ in range(2):
            d.charges.append(sy.Charge("pair", rng.uniform(0.8, 1.5), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                       ("cos", rng.uniform(0.1, 1), rng.uniform(0.1, 0.5), rng.uniform(0, 6.28))))
    return sy.System(h, 0.02, sy.C_AU, doms, name="three spread domains")


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("fp32_ring_i16", 1e-4), ("fp32_ring_fp16", 2e-4),
                                           ("fp32_ring_bf16", 2e-3)])
def test_fused_additions_every_ring_format(precision, tol):
    """8 steps per pass with the own-source lags of steps 2..8 of a block added
    by the inverse x pass (no separate pass over the accumulators), for every
    ring format: every step against the oracle and against one step per
    pass."""
    from paper_2311_15429_amd import plan_for_system
    s = _spread_system()
    p = plan_for_system(s, precision)
    p.set_tuning("lagsum_steps", 8)
    assert p.stats()["fused_additions"] == 1
    assert min(p.info(a, b)[0] for a in range(3) for b in range(3) if a != b) >= 7
    assert p.info(0, 0)[2][0] == 96
    # self windows shorter than a block (lags 0..4): the additions stop at the window
    assert min(p.info(a, a)[1] for a in range(3)) < 7
    p.close()
    L = 2 * 8 + 5
    S = sy.sample_sources(s, range(L + 1))
    got = run_gpu(s, precision, S, tune={"lagsum_steps": 8})
    plain = run_gpu(s, precision, S)
    ref = oracle.potential_full(s, S, range(L + 1))
    worst, worst_d = 0.0, 0.0
    for l in range(L + 1):
        e = rel_err(got[l], ref[l])
        d = rel_err(got[l], plain[l])
        worst, worst_d = max(worst, float(e.max())), max(worst_d, float(d.max()))
        assert np.all(e <= tol), (l, e)
        assert np.all(d <= max(tol / 4, 2e-6)), (l, d)
    log(f"{precision}, fused additions: vs oracle {worst:.2e}, vs one step per pass {worst_d:.2e}")


@pytest.mark.parametrize("dims,pad", [((72, 6, 8), 144), ((96, 6, 8), 192)])
def test_fused_additions_at_the_lengths_of_the_batched_recipe(dims, pad):
    """x-lines of 144 and 192 frequencies (pads of the larger grids of the
    batched recipe), which cross the 256-frequency tiles: 8 steps per pass
    with the own lags added by the inverse x pass, every step against the
    oracle and against one step per pass (FP32)."""
    from paper_2311_15429_amd import plan_for_system
    rng = np.random.default_rng(11)
    h = 0.5
    doms = [sy.Domain(dims, np.array([0.0, 0.0, 0.0])), sy.Domain(dims, np.array([-4.0, 40.0, 3.0]))]
    for d in doms:
        lo = d.origin
        hi = d.origin + h * (np.array(d.dims) - 1)
        for _ in range(2):
            d.charges.append(sy.Charge("pair", rng.uniform(0.8, 1.5), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                       ("cos", rng.uniform(0.1, 1), rng.uniform(0.1, 0.5), rng.uniform(0, 6.28))))
    s = sy.System(h, 0.02, sy.C_AU, doms, name=f"x pad {pad}")
    p = plan_for_system(s, "fp32")
    p.set_tuning("lagsum_steps", 8)
    assert p.stats()["fused_additions"] == 1
    assert p.info(0, 0)[2][0] == pad and p.info(1, 1)[2][0] == pad
    assert min(p.info(0, 1)[0], p.info(1, 0)[0]) >= 7
    p.close()
    L = 2 * 8 + 5
    S = sy.sample_sources(s, range(L + 1))
    got = run_gpu(s, "fp32", S, tune={"lagsum_steps": 8})
    plain = run_gpu(s, "fp32", S)
    ref = oracle.potential_full(s, S, range(L + 1))
    worst, worst_d = 0.0, 0.0
    for l in range(L + 1):
        e = rel_err(got[l], ref[l])
        d = rel_err(got[l], plain[l])
        worst, worst_d = max(worst, float(e.max())), max(worst_d, float(d.max()))
        assert np.all(e <= 2e-5), (l, e)
        assert np.all(d <= 5e-6), (l, d)
    log(f"x pad {pad}, fused additions: vs oracle {worst:.2e}, vs one step per pass {worst_d:.2e}")


def test_blocked_steps_graph_replays_interleaved_with_eager_steps():
    """Batched systems, persistent blocked pass, one graph per phase: replays
    and eager steps in an irregular order, each step against the oracle."""
    from paper_2311_15429_amd import plan_for_system
    from test_gpu_batch import _src, _small_batch, _subsystem
    system = _small_batch(4, 6)
    kb, L = 4, 19
    S = sy.sample_sources(system, range(L + 1))
    p = plan_for_system(system, "fp32", stream=torch.cuda.current_stream())
    p.set_tuning("lagsum_steps", kb)
    p.set_tuning("lagsum_persistent", 1)
    p.bind()
    p.set_green_kernels()
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    buf = [torch.empty_like(o) for o in outs]
    got = {}
    p.push_sources(0, _src(S, 0, p.dims, torch.float32))
    p.retarded_step(0, outs)
    got[0] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    p.capture_step(buf, outs)
    eager = {2, 5, 6, 11, 16, 17}
    for l in range(1, L + 1):
        if l in eager:
            p.push_sources(l, _src(S, l, p.dims, torch.float32))
            p.retarded_step(l, outs)
        else:
            for b, x in zip(buf, _src(S, l, p.dims, torch.float32)):
                b.copy_(x)
            p.launch_step(l)
        got[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    p.close()
    for sid in sorted(set(system.system_id)):
        sub, idx = _subsystem(system, sid)
        ref = oracle.potential_full(sub, [S[i] for i in idx], range(L + 1))
        for l in range(L + 1):
            e = rel_err([got[l][i] for i in idx], ref[l])
            assert np.all(e <= 2e-5), (sid, l, e)
    log(f"blocked graph replays: {len(set(system.system_id))} systems, {L + 1} steps ok")


def test_blocked_steps_state_rules():
    from paper_2311_15429_amd import RpotError, plan_for_system
    from test_gpu_parity import _uneven_system
    s = _uneven_system(8)
    p = plan_for_system(s, "fp32", stream=torch.cuda.current_stream())
    p.set_tuning("lagsum_steps", 4)
    p.bind()
    with pytest.raises(RpotError):
        p.set_tuning("lagsum_steps", 2)                   # after the bind
    p.set_green_kernels()
    S = sy.sample_sources(s, range(3))
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(2):
        p.push_sources(l, [torch.from_numpy(S[n][l].reshape((4,) + p.dims[n])).float().cuda() for n in range(3)])
        p.retarded_step(l, outs)
    with pytest.raises(RpotError):
        p.autotune(iters=1)                               # mid-block (step 2 is phase 1)
    p.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kb", [8, 16])
def test_blocked_steps_config2_full_size_past_the_deepest_lag(kb):
    """Config 2 in FP32 with 8 or 16 steps per pass: sampled points of every
    domain at steps of many phases, the last ones past the deepest lag."""
    from paper_2311_15429_amd import plan_for_system
    from gpu_helpers import cpu_sample_fn
    system = sy.config2(0)
    steps_out = [43, 230, 383, 386, 390, 401]            # phases 2, 5, 6, 1, 5, 0 (of 8)
    rng = np.random.default_rng(11)
    picks = {s: pick_points(d.dims, 24, rng) for s, d in enumerate(system.domains)}
    plan = plan_for_system(system, "fp32", stream=torch.cuda.current_stream())
    plan.set_tuning("lagsum_steps", kb)
    plan.bind()
    plan.set_green_kernels()
    gen = GpuSourceGen(system, plan.dtype)
    outs = [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    sel = [torch.from_numpy(picks[s]).to("cuda") for s in range(8)]
    got = {}
    for l in range(max(steps_out) + 1):
        plan.push_sources(l, gen.step(l))
        plan.retarded_step(l, outs)
        if l in steps_out:
            got[l] = [o.reshape(4, -1)[:, sel[s]].double().cpu().numpy() for s, o in enumerate(outs)]
    torch.cuda.synchronize()
    plan.close()
    fn = cpu_sample_fn(system)
    for l in steps_out:
        ref = [oracle.potential_points(system, s, picks[s], l, fn).T for s in range(8)]
        g, r = np.concatenate(got[l], axis=1), np.concatenate(ref, axis=1)
        e = np.max(np.abs(g - r), axis=1) / np.max(np.abs(r), axis=1)
        log(f"  blocked x{kb}, step {l} (phase {(l - 1) % kb}): max rel err " + " ".join(f"{x:.2e}" for x in e))
        assert np.all(e <= 2e-5), (l, e)
