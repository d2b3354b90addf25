"""Batching: many independent systems with uneven domain counts and grid sizes
in one plan, the persistent lag-sum launch, the graph-captured step and the
autotuner -- each checked against the FP64 oracle or against the eager path."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _small_batch(seed=0, n_systems=10):
    """Systems of 2-4 domains with grids from {6, 8, 10, 12}^3 (pads 12..24,
    radix 2, 3 and 4), h = 0.5, 12-40 bohr apart."""
    rng = np.random.default_rng(seed)
    h = 0.5
    doms, sid = [], []
    for s in range(n_systems):
        nd = int(rng.integers(2, 5))
        ns = [int(rng.choice([6, 8, 10, 12])) for _ in range(nd)]
        cents = []
        for i in range(nd):
            while True:
                c = rng.uniform(-20, 20, size=3)
                if all(np.linalg.norm(c - cj) >= 12 and
                       np.max(np.abs(c - cj)) >= 0.5 * h * (ns[i] + ns[j]) + 2 * h
                       for j, cj in enumerate(cents)):
                    cents.append(c)
                    break
        for i in range(nd):
            d = sy.Domain((ns[i],) * 3, cents[i] + np.array([500.0 * s, 0, 0]) - 0.5 * (ns[i] - 1) * h)
            lo, hi = d.origin, d.origin + h * (ns[i] - 1)
            for _ in range(2):
                d.charges.append(sy.Charge("pair", rng.uniform(0.8, 1.5), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                           ("cos", rng.uniform(0.1, 1), rng.uniform(0.1, 0.5), rng.uniform(0, 6.28))))
            doms.append(d)
            sid.append(s)
    return sy.System(h, 0.02, sy.C_AU, doms, system_id=sid, name=f"batch of {n_systems} systems")


def _subsystem(system, s):
    idx = [i for i, v in enumerate(system.system_id) if v == s]
    return sy.System(system.h, system.dt, system.c, [system.domains[i] for i in idx]), idx


def _plan(system, precision, **tune):
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, precision, stream=torch.cuda.current_stream())
    for k, v in tune.items():
        p.set_tuning(k, v)
    p.bind()
    p.set_green_kernels()
    return p


def _src(S, l, dims, dtype):
    return [torch.from_numpy(np.ascontiguousarray(S[n][l]).reshape((4,) + dims[n])).to("cuda", dtype)
            for n in range(len(dims))]


def _eager(system, precision, S, L, **tune):
    p = _plan(system, precision, **tune)
    outs = [torch.empty((4,) + d, dtype=p.dtype, device="cuda") for d in p.dims]
    res = []
    for l in range(L + 1):
        p.push_sources(l, _src(S, l, p.dims, p.dtype))
        p.retarded_step(l, outs)
        res.append([o.double().cpu().numpy().reshape(4, -1) for o in outs])
    p.close()
    return res


def test_persistent_lagsum_is_bitwise_identical():
    system = _small_batch(1, 6)
    L = 10
    S = sy.sample_sources(system, range(L + 1))
    a = _eager(system, "fp64", S, L, lagsum_persistent=0)
    b = _eager(system, "fp64", S, L, lagsum_persistent=1)
    for l in range(L + 1):
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y), l


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5), ("fp32_ring_i16", 1e-4)])
def test_batched_systems_graph_replay_vs_oracle(precision, tol):
    """One plan for all systems, persistent lag sum, steps >= 1 replayed from a
    captured graph with eager work in between; every system equals its own
    oracle run."""
    system = _small_batch(2, 10)
    L = 14
    S = sy.sample_sources(system, range(L + 1))
    p = _plan(system, precision, lagsum_persistent=1)
    dt = p.dtype
    outs = [torch.empty((4,) + d, dtype=dt, device="cuda") for d in p.dims]
    src_buf = [torch.empty((4,) + d, dtype=dt, device="cuda") for d in p.dims]
    got = {}
    p.push_sources(0, _src(S, 0, p.dims, dt))
    p.retarded_step(0, outs)
    got[0] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    p.capture_step(src_buf, outs)
    for l in range(1, L + 1):
        if l % 3 == 0:            # eager calls interleaved with replays
            p.push_sources(l, _src(S, l, p.dims, dt))
            p.retarded_step(l, outs)
        else:
            for b, x in zip(src_buf, _src(S, l, p.dims, dt)):
                b.copy_(x)
            p.launch_step(l)
        junk = torch.randn(1 << 16, device="cuda").sum()     # unrelated eager work
        got[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
        assert torch.isfinite(junk)
    p.close()
    for s in sorted(set(system.system_id)):
        sub, idx = _subsystem(system, s)
        ref = oracle.potential_full(sub, [S[i] for i in idx], range(L + 1))
        for l in range(L + 1):
            e = rel_err([got[l][i] for i in idx], ref[l])
            assert np.all(e <= tol), (s, l, e)
    log(f"batched {precision}: {len(set(system.system_id))} systems, {len(system.domains)} domains ok")


def test_graph_replay_is_bitwise_identical_to_eager():
    system = _small_batch(3, 4)
    L = 9
    S = sy.sample_sources(system, range(L + 1))
    ref = _eager(system, "fp64", S, L)
    p = _plan(system, "fp64")
    outs = [torch.empty((4,) + d, dtype=torch.float64, device="cuda") for d in p.dims]
    buf = [torch.empty_like(o) for o in outs]
    p.push_sources(0, _src(S, 0, p.dims, torch.float64))
    p.retarded_step(0, outs)
    p.capture_step(buf, outs)
    for l in range(1, L + 1):
        for b, x in zip(buf, _src(S, l, p.dims, torch.float64)):
            b.copy_(x)
        p.launch_step(l)
        torch.cuda.synchronize()
        for o, r in zip(outs, ref[l]):
            assert np.array_equal(o.cpu().numpy().reshape(4, -1), r), l
    p.close()


def test_autotune_selects_a_valid_schedule():
    from test_gpu_parity import _uneven_system
    s = _uneven_system(9)
    L = 8
    S = sy.sample_sources(s, range(L + 1))
    p = _plan(s, "fp32")
    res = p.autotune(iters=2)
    assert res["lagsum_unroll"] in (1, 2, 4) and res["lagsum_persistent"] in (0, 1)
    assert res["fft_lds"] in (2048, 4096, 6144) and not res["cached"]
    assert res["lagsum_ms"] > 0
    assert p.get_tuning("lagsum_unroll") == res["lagsum_unroll"]
    assert p.get_tuning("fft_lds") == res["fft_lds"]
    # one tile per shape class
    assert len(res["fft_lds_per_class"]) == len(p.classes())
    assert all(v in (2048, 4096, 6144) for v in res["fft_lds_per_class"])
    assert [c["fft_lds"] for c in p.classes()] == res["fft_lds_per_class"]
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(L + 1):
        p.push_sources(l, _src(S, l, p.dims, torch.float32))
        p.retarded_step(l, outs)
    got = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    ref = oracle.potential_full(s, S, [L])[0]
    assert np.all(rel_err(got, ref) <= 2e-5)
    p.close()


def test_launch_step_requires_capture_and_order():
    from paper_2311_15429_amd import RpotError
    system = _small_batch(4, 2)
    p = _plan(system, "fp32")
    with pytest.raises(RpotError) as e:
        p.launch_step(1)
    assert e.value.status == "RP_ERR_STATE"
    outs = [torch.zeros((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    p.push_sources(0, outs)
    p.retarded_step(0, outs)
    p.capture_step(outs, outs)
    with pytest.raises(RpotError):
        p.launch_step(2)
    p.launch_step(1)
    torch.cuda.synchronize()
    p.close()


def test_autotune_cache(tmp_path):
    """The second plan of the same shapes takes the stored choice."""
    from test_gpu_parity import _uneven_system
    cache = str(tmp_path / "tune.json")
    s = _uneven_system(11)
    p = _plan(s, "fp32")
    first = p.autotune(iters=1, cache=cache)
    p.close()
    q = _plan(s, "fp32")
    second = q.autotune(iters=1, cache=cache)
    assert second["cached"] and not first["cached"]
    for k in ("lagsum_unroll", "lagsum_persistent", "fft_lds"):
        assert second[k] == first[k] == q.get_tuning(k)
    q.close()


def test_a_different_line_pass_tile_per_shape_class():
    """Every shape class of a batched plan with its own line-pass tile: each
    system still equals its own oracle run."""
    system = _small_batch(2, 11)
    L = 10
    S = sy.sample_sources(system, range(L + 1))
    p = _plan(system, "fp32")
    cls = p.classes()
    assert len(cls) >= 2
    tiles = [(2048, 4096, 6144)[c % 3] for c in range(len(cls))]
    for c, v in enumerate(tiles):
        p.set_class_tuning(c, "fft_lds", v)
    assert [c["fft_lds"] for c in p.classes()] == tiles
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(L + 1):
        p.push_sources(l, _src(S, l, p.dims, torch.float32))
        p.retarded_step(l, outs)
    got = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    ref = oracle.potential_full(system, S, [L])[0]
    e = rel_err(got, ref)
    log(f"per-class tiles {tiles}: rel err {np.array2string(e, precision=2)}")
    assert np.all(e <= 2e-5), e
    p.close()

