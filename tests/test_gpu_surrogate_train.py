"""The trained far-pair surrogate end to end (the gain test): teacher data
from the plain method on other seeds of the same recipe, training by the
library's kernels, then the same workload three ways -- plain, surrogate, and
far pairs dropped -- compared with each other and, at sampled points, with
the FP64 direct-sum oracle.  The surrogate must hold the total error within
1e-4 (per component, relative) where dropping the far pairs does not, and
cut the lag-sum traffic and time."""
import numpy as np
import pytest

import oracle
from gpu_helpers import GpuSourceGen, cpu_sample_fn, log, rel_err
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_DOM, N, BOX, FAR, NL, STEPS = 12, 16, 400.0, 10.0, 64, 1200
TRAIN_SEEDS = range(11, 17)


def recipe(seed):
    """The large surrogate workload's recipe (pairs of Gaussian dipoles in
    boxes placed at random) at test size: 12 boxes of 16^3, 400-bohr volume."""
    return sy.config5(seed, n_dom=N_DOM, n=N, box=BOX)


def _plan(system, mode, audit=()):
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, "fp32", stream=torch.cuda.current_stream())
    if mode != "plain":
        p.surrogate_configure(FAR, n_lags=NL, audit=audit)
    p.bind()
    p.set_green_kernels()
    return p


def test_trained_surrogate_gain():
    from paper_2311_15429_amd import surrogate as S
    X, T = [], []
    for seed in TRAIN_SEEDS:
        system = recipe(seed)
        p = _plan(system, "teacher", audit=range(N_DOM))
        x, t = S.collect_pair_responses(p, GpuSourceGen(system, torch.float32).step, STEPS, every=2)
        X.append(x)
        T.append(t)
        p.close()
    X, T = torch.cat(X), torch.cat(T)
    sur = S.train_surrogate(X, T, NL, iters=10000, batch=1024, max_batch=2048)
    log(f"trained on {X.shape[0]} pair responses, train rel rms {S.relative_rms(sur, X, T):.2e}")
    del X, T

    system = recipe(0)
    gen = GpuSourceGen(system, torch.float32)
    check = [STEPS // 2, STEPS - 1]
    res, lag_ms, lag_bytes, judged = {}, {}, {}, []
    for mode in ("plain", "surrogate", "dropped"):
        p = _plan(system, mode, audit=[0, 5] if mode == "surrogate" else [])
        if mode == "surrogate":
            p.surrogate_attach(sur.mlp, sur.in_scale, sur.out_scale)
        outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
        p.profile_lagsum(True)
        got = {}
        for l in range(STEPS):
            p.push_sources(l, gen.step(l))
            p.retarded_step(l, outs)
            if mode == "surrogate" and l % 100 == 99:      # the judge on sampled steps
                judged.append(p.surrogate_judge(outs, 1e-4))
            if l in check:
                got[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
        ms, n = p.lagsum_time()
        lag_ms[mode], lag_bytes[mode] = ms / n, p.stats()["lagsum_bytes"]
        res[mode] = got
        p.close()
    fell = sum(n for n, _ in judged)
    log(f"judge: {fell} fallbacks, worst error/budget {max(w for _, w in judged):.2f}")
    for l in check:
        e_s = rel_err(res["surrogate"][l], res["plain"][l])
        e_d = rel_err(res["dropped"][l], res["plain"][l])
        log(f"step {l}: surrogate {np.array2string(e_s, precision=2)} dropped {np.array2string(e_d, precision=2)}")
        assert np.all(e_s <= 1e-4), (l, e_s)
        assert np.max(e_d) >= 20 * np.max(e_s)
    # the FP64 direct sum at sampled points of two targets (scale: the plain field)
    l = check[-1]
    fn = cpu_sample_fn(system)
    rng = np.random.default_rng(0)
    for s in (3, 8):
        idx = np.sort(rng.choice(N ** 3, 64, replace=False))
        ref = oracle.potential_points(system, s, idx, l, fn)          # [64][4]
        scale = np.max(np.abs(np.concatenate([r.reshape(4, -1) for r in res["plain"][l]], axis=1)), axis=1)
        got = res["surrogate"][l][s][:, idx].T
        e = np.max(np.abs(got - ref), axis=0) / scale
        assert np.all(e <= 1e-4), (s, e)
    gain_b = lag_bytes["plain"] / lag_bytes["surrogate"]
    gain_t = lag_ms["plain"] / lag_ms["surrogate"]
    log(f"lag sum: {lag_ms['plain']:.3f} -> {lag_ms['surrogate']:.3f} ms/step ({gain_t:.1f}x), bytes {gain_b:.1f}x")
    assert gain_b > 5 and gain_t > 3
    sur.mlp.close()
