"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and plans windows, pads and depths correctly (no GPU needed: planning
makes no HIP call)."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2311_15429_amd import Plan, RpotError, load
from synth import sources as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_AU = 137.036


def test_library_exports_every_declared_symbol():
    lib = load()
    header = open(os.path.join(ROOT, "include", "rpot.h")).read()
    names = set(re.findall(r"^(?:rp_status|const char \*)\s*(rp_[a-z_]+)\s*\(", header, re.M))
    assert {"rp_plan_domains", "rp_set_green_kernels", "rp_push_sources", "rp_retarded_step"} <= names
    for n in names:
        assert hasattr(lib, n), n


def test_config1_windows_pads_depth():
    s = sy.config1(1)
    p = Plan(s.dims, s.origins, s.h, s.dt, s.c, precision="fp64")
    assert p.info(0, 0)[:2] == (0, 5) and p.info(1, 1)[:2] == (0, 5)
    assert p.info(0, 1)[:2] == (8, 15) and p.info(1, 0)[:2] == (8, 15)
    _, _, pad, depth = p.info(0, 1)
    assert pad == (32, 32, 32) and depth == 16
    st = p.stats()
    assert st["n_triples"] == 28
    assert st["n_spectra"] == 6 + 6 + 8           # reversed pair shares its spectra
    assert st["points"] == 2 * 16 ** 3
    assert st["lagsum_bytes"] > 0 and p.workspace_bytes > 0


def _bruteforce_window(dt, dn, h, c, dt_):
    pt = sy.grid_points(dt, h)
    pn = sy.grid_points(dn, h)
    R = np.linalg.norm(pt[:, None, :] - pn[None, :, :], axis=2)
    x = R / (c * dt_)
    return int(np.floor(x.min())), int(np.ceil(x.max()))


@pytest.mark.parametrize("seed", range(6))
def test_windows_match_bruteforce(seed):
    rng = np.random.default_rng(seed)
    h, dt = 0.5, 0.02
    doms = []
    for i in range(3):
        dims = tuple(int(v) for v in rng.integers(1, 6, size=3))
        doms.append(sy.Domain(dims, np.array([9.0 * i, rng.uniform(-3, 3), rng.uniform(-3, 3)])))
    p = Plan([d.dims for d in doms], [d.origin for d in doms], h, dt, C_AU, precision="fp32")
    for s in range(3):
        for n in range(3):
            lo, hi, _, _ = p.info(s, n)
            blo, bhi = _bruteforce_window(doms[s], doms[n], h, C_AU, dt)
            if s == n:
                assert lo == 0 and hi == max(bhi, 1)
            else:
                assert lo == blo and hi == bhi
            rmin, rmax = oracle.box_distance_range(doms[s], doms[n], h)
            assert lo <= rmin / (C_AU * dt) and hi >= rmax / (C_AU * dt)
    for n in range(3):
        assert p.info(0, n)[3] == max(p.info(s, n)[1] for s in range(3)) + 1


def test_pads_are_even_smooth_and_cover_linear_convolution():
    p = Plan([(20, 9, 20), (24, 8, 26), (12, 6, 14)],
             [(0, 0, 0), (15, 3, -2), (-3, 12, 8)], 0.5, 0.02, C_AU)
    pad = p.info(0, 1)[2]
    assert pad == (48, 18, 54)


def test_hartree_limit_plans_single_lag():
    s = sy.config1(1)
    p = Plan(s.dims, s.origins, s.h, s.dt, math.inf, precision="fp64")
    for a in range(2):
        for b in range(2):
            assert p.info(a, b)[:2] == (0, 0)


def test_systems_are_independent():
    dims = [(4, 4, 4)] * 4
    origins = [(0, 0, 0), (10, 0, 0), (0, 0, 0), (10, 0, 0)]   # overlap only across systems
    p = Plan(dims, origins, 0.5, 0.02, C_AU, system_id=[0, 0, 1, 1])
    assert p.info(0, 2)[:2] == (-1, -1)
    assert p.info(0, 1)[0] >= 0 and p.info(2, 3)[0] >= 0


def test_error_paths():
    with pytest.raises(RpotError) as e:
        Plan([(4, 4, 4), (4, 4, 4)], [(0, 0, 0), (1.0, 0, 0)], 0.5, 0.02, C_AU)
    assert e.value.status == "RP_ERR_GEOMETRY"
    with pytest.raises(RpotError) as e:
        Plan(np.zeros((0, 3)), np.zeros((0, 3)), 0.5, 0.02, C_AU)
    assert e.value.status == "RP_ERR_ARG"
    with pytest.raises(RpotError) as e:
        Plan([(4, 4, 4)], [(0, 0, 0)], 0.5, 0.001, C_AU)       # h sqrt3/2 >= c dt
    assert e.value.status == "RP_ERR_UNSUPPORTED"
    with pytest.raises(RpotError) as e:
        Plan([(0, 4, 4)], [(0, 0, 0)], 0.5, 0.02, C_AU)
    assert e.value.status == "RP_ERR_ARG"
    with pytest.raises(RpotError) as e:
        Plan([(300, 4, 4)], [(0, 0, 0)], 0.5, 0.02, C_AU)       # pad above 512
    assert e.value.status == "RP_ERR_UNSUPPORTED"
    p = Plan([(4, 4, 4)], [(0, 0, 0)], 0.5, 0.02, C_AU)
    lib = load()
    assert lib.rp_set_green_kernels(p._h) == 4               # RP_ERR_STATE: not bound
    assert b"not bound" in lib.rp_last_error(p._h)
    assert lib.rp_push_sources(p._h, 0, None) == 4


def test_paper_run_windows_do_not_grow_with_distance():
    """Two C12H4-sized domains (the paper's 20x20x50 a.u. boxes at h = 0.4,
    dt = 1 as): the multi-domain cost (lag window of the cross pair) does not
    grow with their distance, while the history depth follows d/(c dt)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_runs.json")))["c12h4_dimer"]
    h = g["h_au"]
    dt = g["dt_as"] * 1e-18 / json.load(open(os.path.join(ROOT, "tests", "golden", "paper_runs.json")))[
        "atomic_unit_of_time_s"]
    n = [int(round(b / h)) for b in g["box_au"]]
    widths, depths = [], []
    for d in (g["d_sweep_au"][0] + 10, g["d_au"][0], 1000.0, g["d_au"][1]):
        o2 = np.zeros(3)
        o2[g["separation_axis"]] = d
        p = Plan([n, n], [(0, 0, 0), o2], h, dt, C_AU)
        lo, hi, pad, depth = p.info(0, 1)
        widths.append(hi - lo + 1)
        depths.append(depth)
        assert pad == (108, 108, 256)
    assert max(widths) == widths[0] and min(widths) >= 0.5 * widths[0]
    assert depths[-1] > 1300 and depths[0] < 100


def test_fft_tile_knob_host():
    from paper_2311_15429_amd import RpotError, plan_for_system
    p = plan_for_system(sy.config1(1), "fp32")
    assert p.get_tuning("fft_lds") == 2048
    assert plan_for_system(sy.config1(1), "fp64").get_tuning("fft_lds") == 4096
    for v in (4096, 6144, 0):
        p.set_tuning("fft_lds", v)
    with pytest.raises(RpotError) as e:
        p.set_tuning("fft_lds", 1000)
    assert e.value.status == "RP_ERR_ARG"
    # per shape class: config 1 has one class (two 16^3 domains, pad 32^3)
    cls = p.classes()
    assert cls == [{"dims": (16, 16, 16), "pad": (32, 32, 32), "n_domains": 2, "fft_lds": 2048}]
    p.set_class_tuning(0, "fft_lds", 6144)
    assert p.classes()[0]["fft_lds"] == 6144
    p.set_tuning("fft_lds", 4096)                  # the plan's value resets every class
    assert p.classes()[0]["fft_lds"] == 4096
    for bad in ((1, "fft_lds", 2048), (0, "fft_lds", 1000), (0, "lagsum_unroll", 2)):
        with pytest.raises(RpotError) as e:
            p.set_class_tuning(*bad)
        assert e.value.status == "RP_ERR_ARG"
    p.close()


def test_oscillator_create_checks_arguments():
    import ctypes
    from paper_2311_15429_amd import _lib
    from synth import sources as sy
    from paper_2311_15429_amd import plan_for_system
    lib = _lib.load()
    system = sy.config1()
    p = plan_for_system(system, "fp32")

    def create(n_osc, params):
        h = ctypes.c_void_p()
        k = (ctypes.c_int32 * 2)(*n_osc)
        P = np.ascontiguousarray(np.asarray(params, np.float64).reshape(-1, 4))
        code = lib.rp_osc_create(ctypes.byref(h), p._h, k, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return code, h

    ok = [[2.0, 0.1, 1.0, 0.5]] * 3
    code, h = create([2, 1], ok)
    assert code == 0
    nb = ctypes.c_size_t()
    assert lib.rp_osc_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    # steps need a bound workspace
    assert lib.rp_osc_step(h, None, 0.0, None) == 4
    assert b"not bound" in lib.rp_osc_last_error(h)
    lib.rp_osc_destroy(h)
    for n_osc, params in (([300, 0], [[1.0, 0, 1, 0]] * 300),          # too many per domain
                          ([1, 0], [[1.0 / system.dt * 2.5, 0, 1, 0]]),  # omega dt >= 2: unstable
                          ([1, 0], [[1.0, -0.1, 1, 0]]),                 # negative damping
                          ([1, 0], [[float("nan"), 0, 1, 0]])):
        code, h = create(n_osc, params)
        assert code == 1 and not h.value, n_osc
        assert lib.rp_osc_last_error(None)
    p.close()


def test_history_split_plans_rings_and_keeps_the_lag_sum():
    """Two domains far apart: the cross window sits far beyond the self window.
    The split keeps the main ring to the self window, adds one ring per
    source for the cross window, and reads exactly the same lag-sum bytes."""
    from paper_2311_15429_amd import RpotError, plan_for_system
    system = sy.wire_pair(W=8, L=12, d=120, h=0.3, dt=0.01, n_pairs=1)
    plain = plan_for_system(system, "fp32")
    p = plan_for_system(system, "fp32")
    p.history_split(8)
    a, b = plain.stats(), p.stats()
    assert b["split_rings"] == 2 and a["split_rings"] == 0
    assert b["lagsum_bytes"] == a["lagsum_bytes"] and b["n_entries"] == a["n_entries"]
    assert b["ring_bytes"] < 0.5 * a["ring_bytes"] and b["history_bytes"] > 0 and a["history_bytes"] == 0
    for n in range(2):
        self_hi = p.info(n, n)[1]
        cross_lo, cross_hi = p.info(1 - n, n)[:2]
        assert cross_lo - self_hi > 8
        assert p.info(0, n)[3] == self_hi + 1
        assert plain.info(0, n)[3] == cross_hi + 1
    # a gap threshold above the gap keeps one ring; 0 switches the split off
    p.history_split(10 ** 6)
    assert p.stats()["split_rings"] == 0 and p.stats()["ring_bytes"] == a["ring_bytes"]
    p.history_split(8)
    p.history_split(0)
    assert p.stats() == a
    # config 1: self [0, 5], cross [8, 15]; a 2-lag gap is below a threshold of 3
    near = plan_for_system(sy.config1(1), "fp32")
    assert near.info(0, 0)[:2] == (0, 5) and near.info(1, 0)[:2] == (8, 15)
    near.history_split(3)
    assert near.stats()["split_rings"] == 0
    # not with the far-pair surrogate, in either order
    p.history_split(8)
    with pytest.raises(RpotError) as e:
        p.surrogate_configure(3.0)
    assert e.value.status == "RP_ERR_UNSUPPORTED"
    q = plan_for_system(system, "fp32")
    q.surrogate_configure(3.0)
    with pytest.raises(RpotError) as e:
        q.history_split(8)
    assert e.value.status == "RP_ERR_UNSUPPORTED"
    for x in (plain, p, near, q):
        x.close()


def test_history_host_tier_plans_host_rings_and_staging():
    """The host tier moves the real-space rings of a split history to pinned
    host memory: the device keeps one staging snapshot per split source and
    one per split ring, the host buffer holds the rings (window start + 1
    snapshots each), and the lag sum and spectral rings are unchanged.  Since
    the rings no longer cost device memory, a narrow gap that does not pay
    with a device-resident ring does pay with the host tier."""
    from paper_2311_15429_amd import RpotError, plan_for_system, load
    system = sy.wire_pair(W=8, L=12, d=120, h=0.3, dt=0.01, n_pairs=1)
    dev = plan_for_system(system, "fp32")
    dev.history_split(8)
    p = plan_for_system(system, "fp32")
    p.history_split(8)
    assert p.host_history_bytes == 0
    p.history_host(True)
    a, b = dev.stats(), p.stats()
    snap = 4 * int(np.prod(system.domains[0].dims)) * 4
    assert b["split_rings"] == a["split_rings"] == 2
    assert b["lagsum_bytes"] == a["lagsum_bytes"] and b["ring_bytes"] == a["ring_bytes"]
    assert b["history_bytes"] == 2 * 2 * snap            # per source: newest + one split ring
    assert p.host_history_bytes == a["history_bytes"]   # the rings themselves
    assert p.host_history_bytes == sum((p.info(1 - n, n)[0] + 1) * snap for n in range(2))
    assert p.workspace_bytes < dev.workspace_bytes
    p.history_host(False)
    assert p.stats() == a and p.host_history_bytes == 0
    # a one-lag gap: not worth a device-resident ring, worth a host one
    wide = sy.wire_pair(W=24, L=24, d=100, h=0.3, dt=0.01, n_pairs=1)
    q = plan_for_system(wide, "fp32")
    q.history_split(1)
    assert q.stats()["split_rings"] == 0 and q.host_history_bytes == 0
    q.history_host(True)
    assert q.stats()["split_rings"] == 2 and q.host_history_bytes > 0
    # the host tier alone splits nothing
    r = plan_for_system(system, "fp32")
    r.history_host(True)
    assert r.stats()["split_rings"] == 0 and r.host_history_bytes == 0
    # binding errors that need no device
    lib = load()
    h = p._h
    assert lib.rp_bind_history_host(h, None, 0) == 4            # tier off: RP_ERR_STATE
    p.history_host(True)
    assert lib.rp_bind_history_host(h, None, 1 << 30) == 1      # null: RP_ERR_ARG
    assert b"null" in lib.rp_last_error(h)
    buf = ctypes.create_string_buffer(64)
    assert lib.rp_bind_history_host(h, ctypes.addressof(buf), 64) == 3   # too small: RP_ERR_NOMEM
    assert lib.rp_history_host_bytes(h, None) == 1
    assert lib.rp_bind_history_host(r._h, None, 0) == 0         # nothing split: no-op
    for x in (dev, p, q, r):
        x.close()


def test_i16_ring_plans_like_fp16_with_tile_scales():
    """The block-floating-point ring stores 4 bytes per complex value like the
    FP16 ring: the same ring and lag-sum bytes, a workspace larger only by the
    per-tile scales and the FP32 staging of one ingest launch."""
    s = sy.config2(0, n_dom=3, n=16)
    f16 = Plan(s.dims, s.origins, s.h, s.dt, s.c, precision="fp32_ring_fp16")
    i16 = Plan(s.dims, s.origins, s.h, s.dt, s.c, precision="fp32_ring_i16")
    a, b = f16.stats(), i16.stats()
    for key in ("n_triples", "n_entries", "lagsum_bytes", "ring_bytes", "spectra_bytes"):
        assert a[key] == b[key], key
    pad = f16.info(0, 0)[2]
    cpad = -(-pad[0] * pad[1] * (pad[2] // 2 + 1) // 256) * 256
    depth = sum(f16.info(n, n)[3] for n in range(3))
    extra = i16.workspace_bytes - f16.workspace_bytes
    # per-tile scales ([tile][depth][4] floats instead of [depth][4]) plus
    # staging of 3 transforms of [Cpad][4] complex FP32, less the z-pass maxima
    assert 3 * cpad * 32 <= extra <= 3 * cpad * 32 + depth * (cpad // 256) * 16 + 64 * 1024
    # the precision enum ends at RP_FP32_RING_I16
    lib = load()
    h = ctypes.c_void_p()
    dims = np.ascontiguousarray(s.dims, dtype=np.int32)
    org = np.ascontiguousarray(s.origins, dtype=np.float64)
    code = lib.rp_plan_domains(ctypes.byref(h), 3, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               org.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None,
                               ctypes.c_double(s.h), ctypes.c_double(s.dt), ctypes.c_double(s.c), 5, None)
    assert code == 1 and not h.value


def test_target_subset_forms_only_pairs_into_the_targets():
    """rp_plan_targets: only (target <- source) pairs are formed, the pad
    covers the largest target plus the largest source, the updates are the
    targets' points, and every system needs a target."""
    h, dt = 0.5, 0.02
    doms = [sy.Domain((8, 8, 8), np.array([0.0, 0, 0])), sy.Domain((16, 16, 16), np.array([30.0, 0, 0])),
            sy.Domain((8, 8, 8), np.array([0.0, 40.0, 0]))]
    args = ([d.dims for d in doms], [d.origin for d in doms], h, dt, C_AU)
    full = Plan(*args, precision="fp32")
    assert full.info(0, 0)[2] == (32, 32, 32)            # 2 x 16 - 1 -> 32
    sub = Plan(*args, precision="fp32")
    sub.set_targets([0, 2])
    assert sub.info(0, 0)[2] == (24, 24, 24)              # 8 + 16 - 1 -> 24
    assert sub.info(1, 0)[:2] == (-1, -1) and sub.info(0, 1)[:2] == full.info(0, 1)[:2]
    a, b = full.stats(), sub.stats()
    assert b["points"] == 2 * 8 ** 3
    assert b["n_triples"] == sum(full.info(s, n)[1] - full.info(s, n)[0] + 1 for s in (0, 2) for n in range(3))
    assert b["lagsum_bytes"] < a["lagsum_bytes"] and sub.workspace_bytes < full.workspace_bytes
    sub.set_targets(None)                                  # back to every domain
    assert sub.stats() == a
    with pytest.raises(RpotError):
        sub.set_targets([3])
    two = Plan(*args, precision="fp32", system_id=[0, 0, 1])
    with pytest.raises(RpotError):
        two.set_targets([0, 1])                           # system 1 left without a target


def test_split_history_drops_the_lags_before_a_non_target_window():
    """A source that is not a target reaches the targets only from its window
    on: with a split history its own ring keeps lag 0 alone and the window
    sits in a split ring."""
    h, dt = 0.5, 0.02
    doms = [sy.Domain((8, 8, 8), np.array([0.0, 0, 0])), sy.Domain((8, 8, 8), np.array([60.0, 0, 0]))]
    p = Plan([d.dims for d in doms], [d.origin for d in doms], h, dt, C_AU, precision="fp32")
    p.set_targets([0])
    lo, hi = p.info(0, 1)[:2]
    assert lo >= 8 and p.info(1, 1)[3] == hi + 1           # unsplit: lags 0 .. hi of source 1
    plain = p.stats()
    p.history_split(4)
    st = p.stats()
    assert p.info(1, 1)[3] == 1 and st["split_rings"] == 1
    assert st["lagsum_bytes"] == plain["lagsum_bytes"] and st["ring_bytes"] < 0.5 * plain["ring_bytes"]


def test_waves_cover_every_target_once_within_the_budget():
    from paper_2311_15429_amd import waves as W
    s = sy.config4(1, n_systems=5, sizes=(8, 12, 16), n_dom_range=(2, 6))
    big = W.plan_units(s.dims, s.origins, s.system_id, s.h, s.dt, s.c, "fp32", budget=1 << 60)
    sid = np.asarray(s.system_id)
    single = 0
    for k in set(sid.tolist()):
        doms = np.where(sid == k)[0].tolist()
        for t in range(len(doms)):
            p = W._unit_plan(s.dims[doms], s.origins[doms], s.h, s.dt, s.c, "fp32", [t], 8)
            single = max(single, p.workspace_bytes)
            p.close()
    budget = max(single, int(0.6 * max(u.workspace for u in big)))
    units = W.plan_units(s.dims, s.origins, s.system_id, s.h, s.dt, s.c, "fp32", budget=budget)
    waves = W.pack_waves(units, budget)
    assert sorted(t for u in units for t in u.targets) == list(range(len(s.domains)))
    assert len(units) > len(big) and all(u.workspace <= budget for u in units)
    for u in units:                       # a unit's targets share a system and a grid shape
        assert set(sid[u.targets]) == {u.system} and len({s.domains[t].dims for t in u.targets}) == 1
        assert sorted(u.domains) == sorted(np.where(sid == u.system)[0].tolist())
    for w in waves:
        p, doms, targets = W.wave_plan(w, s.dims, s.origins, s.h, s.dt, s.c, "fp32")
        assert w.workspace <= budget and p.workspace_bytes <= w.workspace
        assert p.stats()["points"] == sum(s.domains[doms[t]].n_points for t in targets)
        p.close()


def test_plane_passes_drop_the_z_transformed_array_from_the_fft_bytes():
    """Config 2 (64^3, pads 128^3): with the plane passes the z-transformed
    array (64 x 64 x 65 x 4 complex per domain) is neither written nor read
    back, forward and inverse, with every ring format; an FP64 plan has none."""
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(sy.config2(0), "fp32")
    t1 = 8 * 64 * 64 * 65 * 4 * 8.0
    on = p.stats()
    assert p.get_tuning("fft_plane") == 1
    p.set_tuning("fft_plane", 0)
    off = p.stats()
    assert p.get_tuning("fft_plane") == 0
    assert off["fft_bytes_fwd"] - on["fft_bytes_fwd"] == pytest.approx(2 * t1)
    assert off["fft_bytes_inv"] - on["fft_bytes_inv"] == pytest.approx(2 * t1)
    with pytest.raises(RuntimeError):
        p.set_tuning("fft_plane", 2)
    f16 = plan_for_system(sy.config2(0), "fp32_ring_fp16")
    b16 = f16.stats()
    f16.set_tuning("fft_plane", 0)
    assert f16.stats()["fft_bytes_fwd"] - b16["fft_bytes_fwd"] == pytest.approx(2 * t1)
    assert f16.stats()["fft_bytes_inv"] - b16["fft_bytes_inv"] == pytest.approx(2 * t1)
    d = plan_for_system(sy.config1(0), "fp64")
    s64 = d.stats()
    d.set_tuning("fft_plane", 0)
    assert d.stats()["fft_bytes_inv"] == s64["fft_bytes_inv"]
    for q in (p, f16, d):
        q.close()


def test_fused_additions_are_chosen_only_where_they_are_the_self_pairs():
    """With blocked lag-sum steps the lags m < i of step i of a block are added
    by the inverse x pass only when no cross pair reaches them and the
    register line pass covers the transform; otherwise a separate pass."""
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(sy.config2(0), "fp32")      # cross windows from lag 42 on
    assert p.stats()["fused_additions"] == 0           # one step per pass
    p.set_tuning("lagsum_steps", 8)
    assert p.stats()["fused_additions"] == 1
    p.set_tuning("fft_reg", 0)                         # LDS-staged passes: separate additions
    assert p.stats()["fused_additions"] == 0
    p.set_tuning("fft_reg", 1)
    assert p.stats()["fused_additions"] == 1
    near = plan_for_system(sy.config1(0), "fp32")     # cross windows from lag 8
    near.set_tuning("lagsum_steps", 8)
    assert near.stats()["fused_additions"] == 1
    close = plan_for_system(sy.System(0.5, 0.02, sy.C_AU, [sy.Domain((8, 8, 8), np.zeros(3)),
                                                          sy.Domain((8, 8, 8), np.array([6.0, 0, 0]))]), "fp32")
    close.set_tuning("lagsum_steps", 8)                # cross window from lag 0: not the self pairs alone
    assert close.info(0, 1)[0] <= 6 and close.stats()["fused_additions"] == 0
    for q in (p, near, close):
        q.close()
