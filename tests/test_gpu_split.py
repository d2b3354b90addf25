"""Split history on the GPU: later lag windows in spectral rings of their own,
fed by transforming again the sources kept in a real-space ring (in device
memory, or in pinned host memory streamed back each step).  The lag sum then
reads the same spectra in the same order, so every output is bitwise
identical to the unsplit plan's; and it matches the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, run_gpu
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pair():
    """Two 8x8x12 domains 36 bohr apart: self window [0, 4], cross window about [24, 29]."""
    return sy.wire_pair(W=8, L=12, d=120, h=0.3, dt=0.01, n_pairs=2, seed=4)


def _three():
    """Three uneven domains at 40 and 90 bohr: two far windows per source (those
    of source 2 touch and merge)."""
    rng = np.random.default_rng(9)
    h = 0.3
    doms = [sy.Domain((8, 8, 12), np.array([0.0, 0, 0])), sy.Domain((10, 6, 9), np.array([40.0, 0, 0])),
            sy.Domain((7, 7, 7), np.array([0.0, 0, 90.0]))]
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    return sy.System(h, 0.01, sy.C_AU, doms)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_ring_fp16", "fp32_ring_bf16", "fp32_ring_i16"])
def test_split_history_is_bitwise_identical(precision):
    system = _pair()
    L = 60
    S = sy.sample_sources(system, range(L + 1))
    a = run_gpu(system, precision, S)
    b = run_gpu(system, precision, S, split=8)
    for l in a:
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y), l
    log(f"{precision}: split history bitwise identical over {L + 1} steps")


def test_split_history_three_domains_matches_oracle_fp64():
    from paper_2311_15429_amd import plan_for_system
    system = _three()
    p = plan_for_system(system, "fp64")
    p.history_split(4)
    st = p.stats()
    assert st["split_rings"] == 5, st["split_rings"]   # source 2: its two far windows touch
    p.close()
    L = 80
    steps = [30, 55, L]
    S = sy.sample_sources(system, range(L + 1))
    got = run_gpu(system, "fp64", S, collect=steps, split=4)
    ref = oracle.potential_full(system, S, steps)
    plain = run_gpu(system, "fp64", S, collect=steps)
    for l, r in zip(steps, ref):
        e = rel_err(got[l], r)
        log(f"three domains, split, step {l}: rel err {np.array2string(e, precision=2)}")
        assert np.all(e <= 1e-10), (l, e)
        for x, y in zip(got[l], plain[l]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_ring_fp16", "fp32_ring_i16"])
def test_host_tier_is_bitwise_identical(precision):
    system = _pair()
    L = 60
    S = sy.sample_sources(system, range(L + 1))
    a = run_gpu(system, precision, S, split=8)
    b = run_gpu(system, precision, S, split=8, host=True)
    for l in a:
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y), l
    log(f"{precision}: host tier bitwise identical to the device tier over {L + 1} steps")


def test_host_tier_three_domains_matches_oracle_fp64():
    """Five split rings over three sources, real-space rings in host memory:
    the result is the unsplit plan's, bit for bit, and the oracle's."""
    from paper_2311_15429_amd import plan_for_system
    system = _three()
    p = plan_for_system(system, "fp64")
    p.history_split(4)
    p.history_host(True)
    st = p.stats()
    log(f"three domains, host tier: {st['split_rings']} split rings, host {p.host_history_bytes / 1e6:.2f} MB, "
        f"device staging {st['history_bytes'] / 1e6:.2f} MB")
    assert st["split_rings"] == 5
    p.close()
    L = 80
    steps = [30, 55, L]
    S = sy.sample_sources(system, range(L + 1))
    got = run_gpu(system, "fp64", S, collect=steps, split=4, host=True)
    ref = oracle.potential_full(system, S, steps)
    plain = run_gpu(system, "fp64", S, collect=steps)
    for l, r in zip(steps, ref):
        e = rel_err(got[l], r)
        log(f"three domains, host tier, step {l}: rel err {np.array2string(e, precision=2)}")
        assert np.all(e <= 1e-10), (l, e)
        for x, y in zip(got[l], plain[l]):
            assert np.array_equal(x, y)


def test_host_tier_one_lag_gap_is_bitwise_identical():
    """Self window [0, 9], cross window [11, 23]: a one-lag gap, which only
    the host tier splits (its rings cost no device memory); the split ring
    re-transforms the sources of 11 steps ago, fetched from the host."""
    from paper_2311_15429_amd import plan_for_system
    system = sy.wire_pair(W=24, L=24, d=100, h=0.3, dt=0.01, n_pairs=2, seed=5)
    p = plan_for_system(system, "fp32")
    assert p.info(0, 0)[:2] == (0, 9) and p.info(1, 0)[:2] == (11, 23)
    p.close()
    L = 40
    S = sy.sample_sources(system, range(L + 1))
    a = run_gpu(system, "fp32", S)
    b = run_gpu(system, "fp32", S, split=1, host=True)
    for l in a:
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y), l
    log(f"one-lag gap, host tier: bitwise identical to one ring over {L + 1} steps")


def test_host_tier_needs_a_pinned_buffer():
    import ctypes
    from paper_2311_15429_amd import RpotError, plan_for_system
    system = _pair()
    p = plan_for_system(system, "fp32", stream=torch.cuda.current_stream())
    p.history_split(8)
    p.history_host(True)
    ws = torch.empty(p.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    lib, h = p._lib, p._h
    assert lib.rp_bind_workspace(h, ctypes.c_void_p(ws.data_ptr() + off), ctypes.c_size_t(ws.numel() - off)) == 0
    p._ws = ws
    p.set_green_kernels()
    src = [torch.zeros((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    with pytest.raises(RpotError) as e:
        p.push_sources(0, src)
    assert e.value.status == "RP_ERR_STATE" and "host history" in str(e.value)
    pageable = np.zeros(p.host_history_bytes, dtype=np.uint8)
    assert lib.rp_bind_history_host(h, ctypes.c_void_p(pageable.ctypes.data), ctypes.c_size_t(pageable.size)) == 1
    assert b"pinned" in lib.rp_last_error(h)
    with pytest.raises(ValueError):
        p.bind(host_history=torch.zeros(p.host_history_bytes, dtype=torch.uint8))
    pinned = torch.empty(p.host_history_bytes, dtype=torch.uint8, pin_memory=True)
    assert lib.rp_bind_history_host(h, ctypes.c_void_p(pinned.data_ptr()), ctypes.c_size_t(pinned.numel())) == 0
    p._host_hist = pinned
    out = [torch.empty_like(x) for x in src]
    p.push_sources(0, src)
    p.retarded_step(0, out)
    torch.cuda.synchronize()
    p.close()


@pytest.mark.parametrize("precision,host", [("fp32", False), ("fp32", True), ("fp32_ring_fp16", True),
                                            ("fp32_ring_i16", True)])
def test_split_history_graph_replay_is_bitwise_identical(precision, host):
    from paper_2311_15429_amd import plan_for_system
    system = _pair()
    L = 45
    S = sy.sample_sources(system, range(L + 1))
    src = [[torch.from_numpy(np.ascontiguousarray(S[n][l]).reshape((4,) + tuple(system.domains[n].dims)))
            .to("cuda", torch.float32) for n in range(2)] for l in range(L + 1)]
    res = []
    for capture in ((False, True) if not host else (False, True, "device")):
        p = plan_for_system(system, precision, stream=torch.cuda.current_stream())
        p.history_split(8)
        if host and capture != "device":
            p.history_host(True)
        capture = capture is True
        p.bind()
        p.set_green_kernels()
        outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
        buf = [torch.empty_like(o) for o in outs]
        p.push_sources(0, src[0])
        p.retarded_step(0, outs)
        if capture:
            p.capture_step(buf, outs)
        seq = []
        for l in range(1, L + 1):
            if capture:
                for b, x in zip(buf, src[l]):
                    b.copy_(x)
                p.launch_step(l)
            else:
                p.push_sources(l, src[l])
                p.retarded_step(l, outs)
            torch.cuda.synchronize()
            seq.append([o.cpu().numpy().copy() for o in outs])
        res.append(seq)
        p.close()
    for other in res[1:]:
        for a, b in zip(res[0], other):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,kb,host", [("fp32", 4, False), ("fp32", 8, False), ("fp32_ring_i16", 8, False),
                                               ("fp32", 8, True)])
def test_split_history_with_blocked_steps_is_bitwise_identical(precision, kb, host):
    """With kb lag-sum steps per pass every split ring also keeps the kb - 1
    ages below its window; the split plan still gives the unsplit plan's bits."""
    system = _pair()
    L = 60
    S = sy.sample_sources(system, range(L + 1))
    a = run_gpu(system, precision, S, tune={"lagsum_steps": kb})
    b = run_gpu(system, precision, S, tune={"lagsum_steps": kb}, split=8, host=host)
    for l in a:
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y), l
    log(f"{precision}, {kb} steps per pass{', host tier' if host else ''}: split bitwise identical")
