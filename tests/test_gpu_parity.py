"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Error per step and component: max over every point of every domain of
|P_gpu - P_oracle| / max |P_oracle|.  Bars: 1e-10 in FP64, 2e-5 in FP32.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, run_gpu
from oracle_helpers import Charge, centred
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-10
FP32_TOL = 2e-5


def _samples(system, L):
    return sy.sample_sources(system, range(L + 1))


def _check(system, precision, L, tol, steps=None):
    S = _samples(system, L)
    steps = list(range(L + 1)) if steps is None else steps
    log(f"[{system.name}] {precision}: GPU run of {L + 1} steps")
    got = run_gpu(system, precision, S, collect=steps)
    log(f"[{system.name}] oracle on {len(steps)} steps")
    ref = oracle.potential_full(system, S, steps)
    worst = 0.0
    for i, l in enumerate(steps):
        e = rel_err(got[l], ref[i])
        worst = max(worst, float(e.max()))
        assert np.all(e <= tol), (l, e)
    log(f"[{system.name}] {precision}: worst rel err {worst:.3e}")
    return got, ref


def test_config1_fp64_every_step():
    """2 x 16^3, h = 0.5, 30 bohr apart, dt = 0.02, 40 steps, FP64 <= 1e-10."""
    _check(sy.config1(1), "fp64", 40, FP64_TOL)


def test_config1_fp32_every_step():
    _check(sy.config1(2), "fp32", 40, FP32_TOL)


def _uneven_system(seed=4):
    rng = np.random.default_rng(seed)
    h = 0.5
    doms = [sy.Domain((20, 9, 20), np.array([0.0, 0.0, 0.0])),
            sy.Domain((24, 8, 26), np.array([15.0, 3.0, -2.0])),
            sy.Domain((12, 6, 14), np.array([-3.0, 12.0, 8.0]))]
    for d in doms:
        lo = d.origin
        hi = d.origin + h * (np.array(d.dims) - 1)
        for _ in range(2):
            d.charges.append(sy.Charge("pair", rng.uniform(0.8, 1.5), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                       ("cos", rng.uniform(0.1, 1), rng.uniform(0.1, 0.5), rng.uniform(0, 6.28))))
    return sy.System(h, 0.02, sy.C_AU, doms, name="uneven 3 domains (pads 48x18x54)")


def test_uneven_domains_radix3_ragged_fp32():
    """Three domains of different shapes: pads (48, 18, 54) use radix 2, 3, 4;
    the spectrum length 48*18*28 ends in a partial lag-sum tile."""
    _check(_uneven_system(), "fp32", 24, FP32_TOL)


def test_uneven_domains_fp64():
    _check(_uneven_system(5), "fp64", 16, FP64_TOL)


def test_hartree_limit_c_infinite_fp64():
    s = sy.config1(3)
    s.c = math.inf
    s.name = "config1 geometry, c = inf"
    _check(s, "fp64", 6, FP64_TOL)


def test_degenerate_shapes_fp64():
    """A 1-point domain, a flat (1 x 5 x 7) domain and a line, all coupled."""
    h = 0.5
    doms = [sy.Domain((1, 1, 1), np.array([0.0, 0.0, 0.0])),
            sy.Domain((1, 5, 7), np.array([4.0, -1.0, 0.5])),
            sy.Domain((6, 1, 1), np.array([-5.0, 2.0, 1.0]))]
    rng = np.random.default_rng(9)
    for d in doms:
        d.charges.append(sy.Charge("single", 0.9, d.origin + rng.uniform(-0.3, 0.3, 3), None,
                                   ("cos", 0.7, 0.4, 0.2)))
    s = sy.System(h, 0.02, sy.C_AU, doms, name="degenerate shapes")
    _check(s, "fp64", 10, FP64_TOL)


def test_batched_systems_are_independent_fp64():
    """Two systems in one plan equal two separate oracle runs."""
    a = sy.config1(4)
    b = _uneven_system(6)
    both = sy.System(0.5, 0.02, sy.C_AU, a.domains + b.domains, system_id=[0, 0, 1, 1, 1],
                     name="two systems")
    L = 12
    S = _samples(both, L)
    got = run_gpu(both, "fp64", S)
    ra = oracle.potential_full(a, S[:2], range(L + 1))
    rb = oracle.potential_full(b, S[2:], range(L + 1))
    for l in range(L + 1):
        assert np.all(rel_err(got[l][:2], ra[l]) <= FP64_TOL)
        assert np.all(rel_err(got[l][2:], rb[l]) <= FP64_TOL)


def test_causality_exact_on_gpu():
    """Sources only in domain A: domain B keeps exactly its static potential
    until light from A can arrive, then changes."""
    h, dt = 0.5, 0.02
    A = centred((0, 0, 0), 8, h)
    A.charges.append(Charge("pair", 0.9, np.array([0.5, 0.2, -0.3]), np.array([-0.6, -0.1, 0.4]),
                            ("cos", 0.8, 0.4, 1.1)))
    B = centred((25.0, 3.0, 0.0), 6, h)
    s = sy.System(h, dt, sy.C_AU, [A, B], name="causality")
    rmin, _ = oracle.box_distance_range(B, A, h)
    x = rmin / (sy.C_AU * dt)
    L = int(math.floor(x)) + 3
    got = run_gpu(s, "fp64", _samples(s, L))
    for l in range(L + 1):
        same = np.array_equal(got[l][1], got[0][1])
        assert same == (l <= math.floor(x)), l


def test_time_shift_invariance_bitwise_fp64():
    """Delaying every source by t0 steps delays the output exactly (bitwise)."""
    s = sy.config1(5)
    L, t0 = 20, 7
    S = _samples(s, L)
    Sd = [np.concatenate([np.repeat(x[:1], t0, axis=0), x], axis=0) for x in S]
    a = run_gpu(s, "fp64", S)
    b = run_gpu(s, "fp64", Sd)
    for l in range(L + 1):
        for n in range(2):
            assert np.array_equal(a[l][n], b[l + t0][n]), (l, n)


def test_deterministic_reruns_fp32():
    s = _uneven_system(7)
    S = _samples(s, 8)
    a = run_gpu(s, "fp32", S)
    b = run_gpu(s, "fp32", S)
    for l in a:
        for x, y in zip(a[l], b[l]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,tile", [("fp32", 4096), ("fp32", 6144), ("fp64", 2048), ("fp64", 6144)])
def test_line_pass_tiles(precision, tile):
    """Every line-pass tile (lines staged per block) gives the oracle's result
    on the uneven radix-2/3/4 shapes."""
    s = _uneven_system(10)
    L = 12
    S = _samples(s, L)
    got = run_gpu(s, precision, S, collect=[L], tune={"fft_lds": tile})
    ref = oracle.potential_full(s, S, [L])[0]
    e = rel_err(got[L], ref)
    assert np.all(e <= (FP64_TOL if precision == "fp64" else FP32_TOL)), e


def test_single_domain_fp64():
    """One sub-domain alone: the self pair only (ragged 12 x 10 x 9 grid)."""
    rng = np.random.default_rng(21)
    d = sy.Domain((12, 10, 9), np.array([1.0, -2.0, 0.5]))
    sy._random_pairs(rng, d, 0.5, 2)
    _check(sy.System(0.5, 0.02, sy.C_AU, [d], name="single domain"), "fp64", 12, FP64_TOL)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_largest_fft_length(precision, tol):
    """Two thin 256-point domains: the pads reach 512 along x and z, the
    largest transform length of the library."""
    from paper_2311_15429_amd import plan_for_system
    h = 0.5
    doms = [sy.Domain((256, 4, 4), np.array([0.0, 0.0, 0.0])), sy.Domain((4, 4, 256), np.array([10.0, 8.0, 0.0]))]
    rng = np.random.default_rng(22)
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    s = sy.System(h, 0.02, sy.C_AU, doms, name="pads 512")
    p = plan_for_system(s, precision)
    assert tuple(p.info(0, 0)[2]) == (512, 8, 512)
    p.close()
    _check(s, precision, 8, tol, steps=[4, 8])


@pytest.mark.parametrize("dims_a,dims_b,pz", [((4, 4, 32), (4, 4, 24), 64), ((8, 8, 16), (8, 8, 16), 32),
                                              ((4, 4, 64), (4, 4, 64), 128), ((2, 2, 128), (2, 2, 128), 256),
                                              ((2, 3, 96), (3, 2, 64), 192)])
def test_register_z_passes(dims_a, dims_b, pz):
    """z passes of lengths 32, 64, 128, 192, 256 in registers (contiguous 16-byte
    loads and stores of both real lines of a complex line; sub-domains whose
    z extent is at most half the pad and a multiple of 4 T), beside a class
    that keeps the staged pass: against the oracle, and against the LDS-staged
    passes to FP32 rounding."""
    from paper_2311_15429_amd import plan_for_system
    h = 0.5
    rng = np.random.default_rng(pz)
    doms = [sy.Domain(dims_a, np.zeros(3)), sy.Domain(dims_b, np.array([h * dims_a[0] + 5.0, 1.0, -2.0]))]
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    s = sy.System(h, 0.02, sy.C_AU, doms, name=f"z pad {pz}")
    p = plan_for_system(s, "fp32")
    assert p.info(0, 0)[2][2] == pz
    p.close()
    L = 8
    S = _samples(s, L)
    reg = run_gpu(s, "fp32", S, tune={"fft_reg": 1})
    staged = run_gpu(s, "fp32", S, tune={"fft_reg": 0})
    ref = oracle.potential_full(s, S, [L])[0]
    e = rel_err(reg[L], ref)
    log(f"z pad {pz}: register z passes vs oracle {np.array2string(e, precision=2)}")
    assert np.all(e <= FP32_TOL), e
    for l in range(L + 1):
        d = rel_err(reg[l], staged[l]) if np.any(staged[l][0]) else np.zeros(4)
        assert np.all(d <= 2e-6), (l, d)


@pytest.mark.parametrize("dims_a,dims_b,pad", [((5, 48, 48), (3, 47, 44), 96), ((4, 32, 32), (2, 31, 28), 64),
                                               ((2, 64, 64), (3, 60, 40), 128), ((3, 16, 16), (2, 15, 12), 32),
                                               ((2, 24, 24), (2, 23, 20), 48), ((2, 16, 16), (3, 1, 4), 32)])
@pytest.mark.parametrize("ring", ["fp32", "fp32_ring_fp16"])
def test_plane_passes(dims_a, dims_b, pad, ring):
    """The z and y transforms of an x slice and component in one launch
    (forward: sources to the y-transformed array; inverse: back to the cropped
    potentials), pads 32 to 128, an odd y extent and a z extent below half the
    pad in the second domain (down to one y row and four z points).  With the
    scaled FP16 ring the forward pass also gives one maximum per x slice and
    component for the ring scales.  Against the oracle, and against the
    separate passes: to FP32 rounding (FP32 ring), and within the FP16 ring's
    quantisation of inputs that differ by FP32 rounding."""
    from paper_2311_15429_amd import plan_for_system
    h = 0.5
    rng = np.random.default_rng(pad + len(ring))
    doms = [sy.Domain(dims_a, np.zeros(3)), sy.Domain(dims_b, np.array([h * dims_a[0] + 4.0, 1.0, -2.0]))]
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    s = sy.System(h, 0.02, sy.C_AU, doms, name=f"plane pad {pad}")
    p = plan_for_system(s, "fp32")
    assert tuple(p.info(0, 0)[2][1:]) == (pad, pad)
    p.close()
    L = 8
    S = _samples(s, L)
    plane = run_gpu(s, ring, S, tune={"fft_plane": 1})
    sep = run_gpu(s, ring, S, tune={"fft_plane": 0})
    ref = oracle.potential_full(s, S, [L])[0]
    e = rel_err(plane[L], ref)
    bar = FP32_TOL if ring == "fp32" else 2e-4
    log(f"plane passes, pad {pad}, {ring}: vs oracle {np.array2string(e, precision=2)}")
    assert np.all(e <= bar), e
    agree = 2e-6 if ring == "fp32" else 1e-4
    for l in range(L + 1):
        d = rel_err(plane[l], sep[l]) if np.any(sep[l][0]) else np.zeros(4)
        assert np.all(d <= agree), (l, d)


@pytest.mark.parametrize("dims,pads", [((16, 24, 32), (32, 48, 64)), ((48, 54, 8), (96, 108, 16)),
                                       ((64, 4, 128), (128, 8, 256)), ((32, 128, 8), (64, 256, 16)),
                                       ((96, 6, 8), (192, 12, 16)), ((72, 6, 8), (144, 12, 16))])
def test_i16_ring_quantised_by_the_x_pass(dims, pads):
    """16-bit integer ring: the register x pass quantises each (tile of 256
    frequencies, component) in the same launch (x lengths 32, 64, 96, 128;
    a block's lines cover whole tiles).  Against the staged path (FP32 rows,
    then the separate quantiser) and against the oracle at the ring's bar."""
    h = 0.5
    rng = np.random.default_rng(sum(dims) + 1)
    off = np.array([h * dims[0] + 6.0, 2.0, -1.0])
    doms = [sy.Domain(dims, np.zeros(3)), sy.Domain(dims, off)]
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    s = sy.System(h, 0.02, sy.C_AU, doms, name=f"pads {pads}")
    L = 10
    S = _samples(s, L)
    fused = run_gpu(s, "fp32_ring_i16", S, tune={"fft_reg": 1})
    staged = run_gpu(s, "fp32_ring_i16", S, tune={"fft_reg": 0})
    ref = oracle.potential_full(s, S, [L])[0]
    e = rel_err(fused[L], ref)
    log(f"pads {pads}, I16 ring quantised by the x pass: rel err vs oracle {np.array2string(e, precision=2)}")
    assert np.all(e <= 1e-4), e
    for l in range(1, L + 1):
        d = rel_err(fused[l], staged[l])
        assert np.all(d <= 2e-5), (l, d)


@pytest.mark.parametrize("dims,pads", [((16, 24, 32), (32, 48, 64)), ((48, 54, 8), (96, 108, 16)),
                                       ((64, 4, 128), (128, 8, 256)), ((32, 128, 8), (64, 256, 16)),
                                       ((96, 6, 8), (192, 12, 16)), ((6, 96, 8), (12, 192, 16)),
                                       ((72, 6, 8), (144, 12, 16)), ((24, 6, 8), (48, 12, 16)),
                                       ((128, 6, 8), (256, 12, 16))])
def test_fixed_length_transforms_fp32(dims, pads):
    """Pads that reach every transform length with a compile-time FP32 kernel
    (x: 32, 48, 64, 96, 128, 256; y: 48, 108, 256; z: 64, 256) and some without
    one (8, 12, 16, 144, 192).  The register-resident line passes (lengths 32, 48,
    64, 96, 128, 144, 192, 256) and the LDS-staged passes at the 2048 and 4096 tiles
    give the oracle's result, and both agree with the run-time kernel of the
    6144 tile to FP32 rounding."""
    from paper_2311_15429_amd import plan_for_system
    h = 0.5
    rng = np.random.default_rng(sum(dims))
    off = np.array([h * dims[0] + 6.0, 2.0, -1.0])
    doms = [sy.Domain(dims, np.zeros(3)), sy.Domain(dims, off)]
    for d in doms:
        sy._random_pairs(rng, d, h, 2)
    s = sy.System(h, 0.02, sy.C_AU, doms, name=f"pads {pads}")
    p = plan_for_system(s, "fp32")
    assert tuple(p.info(0, 0)[2]) == pads
    p.close()
    L = 10
    S = _samples(s, L)
    runs = {tile: run_gpu(s, "fp32", S, tune={"fft_reg": 0, "fft_lds": tile}) for tile in (2048, 4096, 6144)}
    runs["reg"] = run_gpu(s, "fp32", S, tune={"fft_reg": 1})
    ref = oracle.potential_full(s, S, [L])[0]
    for tile in (2048, 4096, "reg"):
        e = rel_err(runs[tile][L], ref)
        log(f"pads {pads}, line pass {tile}: rel err vs oracle {np.array2string(e, precision=2)}")
        assert np.all(e <= FP32_TOL), (tile, e)
        for l in range(L + 1):
            d = rel_err(runs[tile][l], runs[6144][l]) if np.any(runs[6144][l][0]) else np.zeros(4)
            assert np.all(d <= 2e-6), (tile, l, d)
