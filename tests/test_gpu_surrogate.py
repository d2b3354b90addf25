"""Far-pair surrogate on the GPU, through the C-ABI: network inputs and plain
pair responses against the FP64 oracle, far pairs left out when no network is
attached, the judge's fallback to the plain lag sum, and graph replay."""
import numpy as np
import pytest

import oracle
from oracle import surrogate_ref as sr
from oracle.ref import contrib, self_cell_c1
from gpu_helpers import GpuSourceGen, log, rel_err
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_LAGS = 16
FAR = 3.0


def far_system(seed=0, n=8, h=0.5):
    """Five 8^3 boxes: a close pair (0, 1) and three boxes 40-70 bohr away."""
    rng = np.random.default_rng(seed)
    cents = [(0, 0, 0), (8, 0, 0), (40, 5, -3), (-10, 45, 12), (25, -30, 50)]
    doms = []
    for c in cents:
        d = sy.Domain((n, n, n), np.array(c, float) - 0.5 * (n - 1) * h)
        lo, hi = d.origin, d.origin + h * (n - 1)
        for _ in range(2):
            d.charges.append(sy.Charge("pair", rng.uniform(0.8, 1.2), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                       ("cos", rng.uniform(0.3, 1.0), rng.uniform(0.5, 2.0), rng.uniform(0, 6.3))))
        doms.append(d)
    return sy.System(h, 0.02, sy.C_AU, doms)


def make_plan(system, audit=None, precision="fp32", steps=1):
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, precision, stream=torch.cuda.current_stream())
    if steps > 1:
        p.set_tuning("lagsum_steps", steps)
    p.surrogate_configure(FAR, n_lags=N_LAGS, audit=range(len(system.domains)) if audit is None else audit)
    p.bind()
    p.set_green_kernels()
    return p


def run(p, gen, L, outs=None, each=None):
    outs = outs or [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(L + 1):
        p.push_sources(l, gen.step(l))
        p.retarded_step(l, outs)
        if each:
            each(l, outs)
    return outs


def pair_field(system, S, s, n, l):
    """Oracle: dynamic contribution [4][N_s] of source n to target s at step l."""
    h = system.h
    pts = sr.grid_points(system.domains[s], h)
    out = np.zeros((len(pts), 4))
    hist = S[n]
    contrib(pts, None, system.domains[n], h, hist[1:], 1, hist.shape[0] - 1, hist[0], l * system.dt, system.dt,
            system.c, True, self_cell_c1(), out)
    return out.T.copy()


def test_features_match_oracle():
    system = far_system(1)
    L = 40
    S = sy.sample_sources(system, range(L + 1))
    p = make_plan(system)
    run(p, GpuSourceGen(system, torch.float32), L)
    x = p.surrogate_features().double().cpu().numpy()
    pairs = p.surrogate_pairs()
    worst = 0.0
    for f, (s, n) in enumerate(zip(pairs["target"], pairs["source"])):
        want = sr.features(system, S, int(s), int(n), L, N_LAGS)
        mom = slice(0, 6 * N_LAGS * 22)
        scale = np.max(np.abs(want[mom]))
        assert scale > 0
        e = np.max(np.abs(x[f, mom] - want[mom])) / scale
        worst = max(worst, e)
        assert np.allclose(x[f, -2:], want[-2:], rtol=1e-6, atol=1e-7)
    assert worst < 2e-5, worst
    log(f"features: {len(pairs['target'])} far pairs, worst rel err {worst:.2e}")
    p.close()


def test_pair_response_matches_oracle():
    system = far_system(2)
    L = 36
    S = sy.sample_sources(system, range(L + 1))
    p = make_plan(system)
    run(p, GpuSourceGen(system, torch.float32), L)
    coef, resid = p.surrogate_pair_response()
    coef, resid = coef.double().cpu().numpy(), resid.double().cpu().numpy()
    pairs = p.surrogate_pairs()
    aud = np.nonzero(pairs["audited"])[0]
    worst = 0.0
    for v, f in enumerate(aud):
        s, n = int(pairs["target"][f]), int(pairs["source"][f])
        F = pair_field(system, S, s, n, L)
        a = sr.frame_fit(system, s, n, F)
        G = sr.frame_synth(system, s, n, a)
        e = np.max(np.abs(coef[v] - a.ravel())) / np.max(np.abs(a))
        worst = max(worst, e)
        fmax = np.max(np.abs(F), axis=1)
        assert np.allclose(resid[v, 4:], fmax, rtol=1e-4, atol=1e-6 * fmax.max())
        fit = np.max(np.abs(F - G), axis=1)
        assert np.all(np.abs(resid[v, :4] - fit) <= 1e-4 * fmax.max() + 1e-3 * fit)
    assert worst < 1e-4, worst
    log(f"pair responses: {len(aud)} audited pairs, worst coefficient rel err {worst:.2e}")
    p.close()


def test_far_pairs_dropped_without_network():
    """No network attached: the output is the full result minus the far pairs'
    dynamic terms (their static terms stay)."""
    system = far_system(3)
    L = 30
    S = sy.sample_sources(system, range(L + 1))
    p = make_plan(system, audit=[])
    outs = run(p, GpuSourceGen(system, torch.float32), L)
    got = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    ref = oracle.potential_full(system, S, [L])[0]
    pairs = p.surrogate_pairs()
    for s, n in zip(pairs["target"], pairs["source"]):
        ref[int(s)] = ref[int(s)] - pair_field(system, S, int(s), int(n), L)
    e = rel_err(got, ref)
    assert np.all(e <= 2e-5), e
    p.close()


def _random_mlp(n_in, n_far, scale=0.05, seed=0):
    from paper_2311_15429_amd.mlp import Mlp
    m = Mlp(n_in, 32, 80, max(n_far, 1))
    g = torch.Generator().manual_seed(seed)
    m.set_params(torch.randn(m.n_params, generator=g) * scale)
    return m


@pytest.mark.parametrize("steps", [1, 4])
def test_judge_falls_back_and_then_matches_the_plain_method(steps):
    """A loose judge keeps every pair on the network, a tight one sends every
    audited pair back to the plain lag sum; from then on the output is the
    oracle's.  With 4 lag-sum steps per pass both judgements fall on the last
    step of a block and the blocked schedules take the pairs over."""
    system = far_system(4)
    L, Lj = 34, 24
    S = sy.sample_sources(system, range(L + 1))
    p = make_plan(system, steps=steps)
    info = p.surrogate_info()
    mlp = _random_mlp(info["n_in"], info["n_far"])
    p.surrogate_attach(mlp, np.full(22, 1.0, np.float32), np.full(80, 1e-3, np.float32))
    gen = GpuSourceGen(system, torch.float32)
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    got = {}
    for l in range(L + 1):
        p.push_sources(l, gen.step(l))
        p.retarded_step(l, outs)
        if l == Lj - steps:
            nf, worst = p.surrogate_judge(outs, 1e3)       # loose: nobody falls back
            assert nf == 0 and 0 < worst < 1
        if l == Lj:
            nf, worst = p.surrogate_judge(outs, 1e-6)      # tight: every audited pair falls back
            assert nf == info["n_far"] and worst > 1
            assert p.surrogate_pairs()["fallen_back"].all()
        if l >= Lj:
            got[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    ref = oracle.potential_full(system, S, sorted(got))
    for (l, g), r in zip(sorted(got.items()), ref):
        e = rel_err(g, r)
        assert np.all(e <= 2e-5), (l, e)
    log(f"judge: {info['n_far']} pairs fell back; steps {Lj}..{L} match the oracle")
    p.surrogate_attach(None)
    p.close()
    mlp.close()


def test_graph_replay_with_surrogate_is_bitwise_identical():
    system = far_system(5)
    L = 20
    gen = GpuSourceGen(system, torch.float32)
    res = []
    for capture in (False, True):
        p = make_plan(system, audit=[2])
        info = p.surrogate_info()
        mlp = _random_mlp(info["n_in"], info["n_far"], seed=7)
        p.surrogate_attach(mlp, np.full(22, 0.5, np.float32), np.full(80, 1e-3, np.float32))
        outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
        buf = [torch.empty_like(o) for o in outs]
        p.push_sources(0, gen.step(0))
        p.retarded_step(0, outs)
        if capture:
            p.capture_step(buf, outs)
        seq = []
        for l in range(1, L + 1):
            if capture:
                for b, x in zip(buf, gen.step(l)):
                    b.copy_(x)
                p.launch_step(l)
            else:
                p.push_sources(l, gen.step(l))
                p.retarded_step(l, outs)
            torch.cuda.synchronize()
            seq.append([o.cpu().numpy().copy() for o in outs])
        res.append(seq)
        p.surrogate_attach(None)
        p.close()
        mlp.close()
    for a, b in zip(*res):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def _box_synth_from_nodes(system, s, F_nodes):
    """Oracle side of the multipole path: least-squares fit of node values
    [4][64] on the 4 x 4 x 4 nodes, synthesised on the target grid."""
    nodes = np.array([-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0])
    xi = np.array([[nodes[t >> 4], nodes[(t >> 2) & 3], nodes[t & 3]] for t in range(64)])
    Bn = sr.basis(xi)
    coef, *_ = np.linalg.lstsq(Bn, F_nodes.T, rcond=None)
    return (sr.basis(sr.box_coords(system.domains[s])) @ coef).T


def test_multipole_terms_match_the_oracle_formula():
    system = far_system(7)
    L = 60
    S = sy.sample_sources(system, range(L + 1))
    gen = GpuSourceGen(system, torch.float32)
    res = {}
    for mode in ("multipole", "dropped"):
        p = make_plan(system, audit=[])
        if mode == "multipole":
            p.surrogate_multipole(True)
        outs = run(p, gen, L)
        res[mode] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
        pairs = p.surrogate_pairs()
        p.close()
    h = system.h
    worst = 0.0
    for s in sorted(set(int(t) for t in pairs["target"])):
        dom = system.domains[s]
        hw = 0.5 * h * (np.array(dom.dims) - 1)
        nodes = np.array([-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0])
        xi = np.array([[nodes[t >> 4], nodes[(t >> 2) & 3], nodes[t & 3]] for t in range(64)])
        pts = sr.box_centre(dom, h) + xi * hw
        want = np.zeros((4, dom.n_points))
        for t_, n in zip(pairs["target"], pairs["source"]):
            if int(t_) == s:
                want += _box_synth_from_nodes(system, s, sr.multipole_field(system, S, s, int(n), L, pts))
        got = res["multipole"][s] - res["dropped"][s]
        scale = np.max(np.abs(want), axis=1)
        e = np.max(np.abs(got - want), axis=1) / scale
        worst = max(worst, float(e.max()))
        assert np.all(e <= 2e-4), (s, e)
    # and the far terms bring the total close to the direct sum
    ref = oracle.potential_full(system, S, [L])[0]
    e_mp = rel_err(res["multipole"], ref)
    e_dr = rel_err(res["dropped"], ref)
    log(f"multipole: formula match {worst:.1e}; total rel err {np.array2string(e_mp, precision=2)} "
        f"vs far pairs left out {np.array2string(e_dr, precision=2)}")
    assert np.max(e_mp) <= np.max(e_dr) / 10


def _node_points(system, s):
    dom = system.domains[s]
    hw = 0.5 * system.h * (np.array(dom.dims) - 1)
    nodes = np.array([-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0])
    xi = np.array([[nodes[t >> 4], nodes[(t >> 2) & 3], nodes[t & 3]] for t in range(64)])
    return sr.box_centre(dom, system.h) + xi * hw


def test_multipole_response_matches_the_oracle():
    """Frame coefficients of the multipole terms of the audited pairs at the
    last completed step: the oracle's multipole field at the nodes, fitted to
    the box basis, synthesised and fitted to the frame basis."""
    system = far_system(8)
    L = 50
    S = sy.sample_sources(system, range(L + 1))
    p = make_plan(system)
    run(p, GpuSourceGen(system, torch.float32), L)
    got = p.surrogate_multipole_response().double().cpu().numpy()
    pairs = p.surrogate_pairs()
    aud = np.nonzero(pairs["audited"])[0]
    worst = 0.0
    for v, f in enumerate(aud):
        s, n = int(pairs["target"][f]), int(pairs["source"][f])
        F = _box_synth_from_nodes(system, s, sr.multipole_field(system, S, s, n, L, _node_points(system, s)))
        want = sr.frame_fit(system, s, n, F).ravel()
        e = np.max(np.abs(got[v] - want)) / np.max(np.abs(want))
        worst = max(worst, e)
    log(f"multipole response: {len(aud)} audited pairs, worst rel err {worst:.1e}")
    assert worst < 2e-4, worst
    p.close()


def test_hybrid_adds_the_network_to_the_multipole_terms():
    system = far_system(9)
    L = 40
    gen = GpuSourceGen(system, torch.float32)
    res = {}
    info = None
    for mode in ("dropped", "multipole", "network", "hybrid0", "hybrid"):
        p = make_plan(system, audit=[])
        info = p.surrogate_info()
        mlp = None
        if mode in ("network", "hybrid"):
            mlp = _random_mlp(info["n_in"], info["n_far"], scale=0.05, seed=11)
        elif mode == "hybrid0":
            from paper_2311_15429_amd.mlp import Mlp
            mlp = Mlp(info["n_in"], 32, 80, info["n_far"])
            mlp.set_params(torch.zeros(mlp.n_params))
        if mode.startswith("hybrid"):
            p.surrogate_multipole("hybrid")
        elif mode == "multipole":
            p.surrogate_multipole(True)
        if mlp is not None:
            p.surrogate_attach(mlp, np.full(22, 1.0, np.float32), np.full(80, 1e-2, np.float32))
        outs = run(p, gen, L)
        res[mode] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
        p.surrogate_attach(None)
        p.close()
        if mlp is not None:
            mlp.close()
    for a, b in zip(res["hybrid0"], res["multipole"]):
        assert np.array_equal(a, b)
    want = [m + w - d for m, w, d in zip(res["multipole"], res["network"], res["dropped"])]
    e = rel_err(res["hybrid"], want)
    net_part = rel_err(res["network"], res["dropped"])
    log(f"hybrid = multipole + network: rel err {np.array2string(e, precision=2)}; "
        f"network part {np.array2string(net_part, precision=2)}")
    assert np.all(net_part > 1e-5), net_part
    assert np.all(e <= 1e-3 * net_part + 1e-7), (e, net_part)


def test_multipole_response_leaves_the_judged_step_intact():
    """The judge corrects a step with that step's own far-pair terms: asking
    for the multipole response first must not change what it does."""
    system = far_system(10)
    L = 30
    res = []
    for query in (False, True):
        gen = GpuSourceGen(system, torch.float32)
        p = make_plan(system)
        info = p.surrogate_info()
        mlp = _random_mlp(info["n_in"], info["n_far"], scale=0.05, seed=3)
        p.surrogate_multipole("hybrid")
        p.surrogate_attach(mlp, np.full(22, 1.0, np.float32), np.full(80, 1e-2, np.float32))
        outs = run(p, gen, L)
        if query:
            p.surrogate_multipole_response()
        nf, _ = p.surrogate_judge(outs, 1e-6)
        assert nf == info["n_far"]
        res.append([o.cpu().numpy().copy() for o in outs])
        p.surrogate_attach(None)
        p.close()
        mlp.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_readmission_restores_the_far_terms():
    """Every audited pair falls back under a tiny tolerance, then returns under
    a loose one with a re-admission factor: from then on the outputs are those
    of a run that never fell back, bit for bit."""
    system = far_system(11)
    L, Lf, Lb = 60, 42, 47   # after every far field has arrived (farthest pair: 33 lags)
    res = []
    for judge in (False, True):
        gen = GpuSourceGen(system, torch.float32)
        p = make_plan(system)
        n_far = p.surrogate_info()["n_far"]
        p.surrogate_multipole(True)
        outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
        seq = {}
        for l in range(L + 1):
            p.push_sources(l, gen.step(l))
            p.retarded_step(l, outs)
            if judge and l == Lf:
                nf, _ = p.surrogate_judge(outs, 1e-12)
                assert nf == n_far and p.last_readmitted == 0
                assert p.surrogate_pairs()["fallen_back"].all()
            if judge and l == Lb:
                p.surrogate_readmit(0.5)
                nf, _ = p.surrogate_judge(outs, 1e3)
                assert nf == 0 and p.last_readmitted == n_far
                assert not p.surrogate_pairs()["fallen_back"].any()
            if l > Lb:
                seq[l] = [o.cpu().numpy().copy() for o in outs]
        res.append(seq)
        p.close()
    for l in res[0]:
        for x, y in zip(res[0][l], res[1][l]):
            assert np.array_equal(x, y), l


def test_training_data_calls_match_their_definitions():
    """rp_surrogate_teacher rows are the audited pairs' features and their
    plain responses times the pair distance (minus the multipole terms with
    residual); the scales, the scaling and the network's relative RMS equal
    their definitions evaluated in numpy (FP64)."""
    from paper_2311_15429_amd import surrogate as S
    system = far_system(3)
    p = make_plan(system, audit=[2, 3])
    run(p, GpuSourceGen(system, torch.float32), 30)
    info, pairs = p.surrogate_info(), p.surrogate_pairs()
    aud = np.nonzero(pairs["audited"])[0]
    assert info["n_audited"] == len(aud) > 0
    feats = p.surrogate_features().cpu().numpy()
    coef, _ = p.surrogate_pair_response()
    coef = coef.cpu().numpy()
    mpole = p.surrogate_multipole_response().cpu().numpy()
    X = torch.empty((len(aud), info["n_in"]), dtype=torch.float32, device="cuda")
    T = torch.empty((len(aud), 80), dtype=torch.float32, device="cuda")
    lib = S._lib.load()
    for residual in (0, 1):
        assert lib.rp_surrogate_teacher(p._h, S._ptr(X), S._ptr(T), residual) == 0
        torch.cuda.synchronize()
        assert np.array_equal(X.cpu().numpy(), feats[aud])
        want = (coef - (mpole if residual else 0.0)) * pairs["dist"][aud][:, None]
        got = T.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want)), residual
    p.close()

    # scales and scaling on random rows (two lags: n_in = 266)
    rng = np.random.default_rng(0)
    nl, n = 2, 300
    x = (rng.normal(size=(n, 132 * nl + 2)) * rng.uniform(0.1, 10, size=132 * nl + 2)).astype(np.float32)
    x[:, 5::22] = 0.0                                          # an all-zero moment gets scale 1
    t = (rng.normal(size=(n, 80)) * np.repeat([1.0, 3.0, 0.5, 2.0], 20)).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    ins, outs = S.feature_scales(xd, td, nl)
    h = x[:, :22 * nl].astype(np.float64).reshape(n, nl, 22)
    rms_in = np.sqrt(np.mean(h ** 2, axis=(0, 1)))
    want_in = np.where(rms_in > 0, 1.0 / np.where(rms_in > 0, rms_in, 1.0), 1.0)
    rms_out = np.sqrt(np.mean(t.astype(np.float64).reshape(n, 4, 20) ** 2, axis=(0, 2)))
    assert np.allclose(ins, want_in, rtol=1e-6) and ins[5] == 1.0
    assert np.allclose(outs, np.repeat(rms_out, 20), rtol=1e-6)
    S.scale_data(xd, td, ins, outs, nl)
    sx = np.ones(132 * nl + 2, np.float32)
    sx[:132 * nl] = np.tile(ins, 6 * nl)
    assert np.allclose(xd.cpu().numpy(), x * sx, rtol=1e-6)
    assert np.allclose(td.cpu().numpy(), t / outs, rtol=1e-6)

    # relative RMS of a small network on the raw rows
    from paper_2311_15429_amd.mlp import Mlp
    net = Mlp(132 * nl + 2, 16, 80, 64)
    net.set_params(torch.from_numpy(rng.normal(scale=0.05, size=net.n_params).astype(np.float32)))
    sur = S.TrainedSurrogate(net, ins, outs, nl, [])
    xs = torch.from_numpy(x * sx).cuda()
    y = torch.cat([net.forward(xs[i:i + 64]) for i in range(0, n, 64)]).double().cpu().numpy() * outs
    want = np.sqrt(np.sum((y - t) ** 2) / np.sum(t.astype(np.float64) ** 2))
    got = S.relative_rms(sur, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    assert abs(got - want) <= 1e-6 * want, (got, want)
    log(f"training-data calls: teacher rows {len(aud)}, relative RMS {got:.4f}")
