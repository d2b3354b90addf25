"""The coupled propagation loop on the GPU (rp_osc_* through the C-ABI):
oscillator sources driven by the path's potentials, against the FP64 loop of
the oracle; and one projection / update / synthesis step at larger, ragged
sizes and over more domains than one launch holds, against the oracle's
projection and synthesis."""
import math

import numpy as np
import pytest

from oracle import coupled_ref as cr
from gpu_helpers import log
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _osc_system(seed=0, n=8, h=0.4, dt=0.02, dist=6.0, n_pairs=2):
    rng = np.random.default_rng(seed)
    doms = []
    for c in ((0.0, 0.0, 0.0), (0.0, dist, 0.0)):
        d = sy.Domain((n, n, n), np.asarray(c) - 0.5 * h * (n - 1))
        sy._random_pairs(rng, d, h, n_pairs)
        doms.append(d)
    system = sy.System(h, dt, sy.C_AU, doms)
    params = []
    for i, d in enumerate(doms):
        p = np.zeros((n_pairs, 4))
        p[:, 0] = rng.uniform(2.0, 8.0, n_pairs)
        p[:, 1] = 0.1
        p[:, 2] = 1.0 if i == 0 else 20.0
        if i == 0:
            p[:, 3] = [ch.cp[2] - ch.cm[2] for ch in d.charges]
        params.append(p)
    return system, params


def _pulse(t, T_env=0.8, w=4.0):
    return 5.0 * math.sin(math.pi * t / T_env) ** 2 * math.sin(w * t) if t < T_env else 0.0


def _gpu_loop(system, bases, params, L, precision, steps=1):
    from paper_2311_15429_amd import Oscillators, plan_for_system
    plan = plan_for_system(system, precision, stream=torch.cuda.current_stream())
    if steps > 1:
        plan.set_tuning("lagsum_steps", steps)
    plan.bind()
    plan.set_green_kernels()
    dt_ = plan.dtype
    bt = [torch.from_numpy(b).to("cuda", dt_).contiguous() for b in bases]
    osc = Oscillators(plan, bt, params)
    src = [torch.empty((4,) + d, dtype=dt_, device="cuda") for d in plan.dims]
    nxt = [torch.empty_like(s) for s in src]
    outs = [torch.empty_like(s) for s in src]
    osc.sources(src)
    qs, qds = [], []
    for l in range(L + 1):
        plan.push_sources(l, src)
        plan.retarded_step(l, outs)
        q, qd, _, _ = osc.state()
        qs.append(q)
        qds.append(qd)
        osc.step(outs, _pulse(l * system.dt), nxt)
        src, nxt = nxt, src
    res = np.array(qs), np.array(qds), [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    osc.close()
    plan.close()
    return res


@pytest.mark.parametrize("precision,tol,steps", [("fp64", 1e-9, 1), ("fp32", 2e-4, 1), ("fp32", 2e-4, 8)])
def test_coupled_loop_matches_the_oracle(precision, tol, steps):
    """The sources of step l + 1 come from the potentials of step l; with 8
    lag-sum steps per pass every step still returns its own potential."""
    system, params = _osc_system(1)
    bases = [sy.pair_shapes(d, system.h, system.c) for d in system.domains]
    L = 60
    rec = cr.run_loop(system, bases, params, _pulse, L)
    q, qd, _ = _gpu_loop(system, bases, params, L, precision, steps)
    want_q = np.concatenate(rec["q"], axis=1)
    want_qd = np.concatenate(rec["qdot"], axis=1)
    # domain 1 is driven only through the potentials (each oscillator is
    # compared on its own scale below)
    assert np.max(np.abs(want_q[:, 2:])) > 1e-3 * np.max(np.abs(want_q[:, :2]))
    for got, want, name in ((q, want_q, "q"), (qd, want_qd, "qdot")):
        e = np.max(np.abs(got - want), axis=0) / np.max(np.abs(want), axis=0)
        log(f"{precision} coupled loop, {L} steps, {steps} per pass: {name} rel err per oscillator "
            f"{np.array2string(e, precision=2)}")
        assert np.all(e <= tol), (name, e)


def _one_step_case(doms, K, h=0.3, dt=0.01, seed=5):
    """Random potentials and state on domains `doms`; one rp_osc_step against
    the oracle's projection, update and synthesis (FP32 path)."""
    from paper_2311_15429_amd import Oscillators, plan_for_system
    rng = np.random.default_rng(seed)
    system = sy.System(h, dt, sy.C_AU, doms)
    bases, params = [], []
    for d, k in zip(doms, K):
        sy._random_pairs(rng, d, h, k)
        bases.append(sy.pair_shapes(d, h, system.c) if k else None)
        params.append(np.column_stack([rng.uniform(1, 10, k), rng.uniform(0, 1, k), rng.uniform(0.5, 2, k),
                                       rng.uniform(-1, 1, k)]))
    plan = plan_for_system(system, "fp32", stream=torch.cuda.current_stream())
    bt = [None if b is None else torch.from_numpy(b).to("cuda", torch.float32).contiguous() for b in bases]
    osc = Oscillators(plan, bt, params)
    tot = sum(K)
    q0, qd0 = rng.normal(size=tot), rng.normal(size=tot)
    osc.set_state(q0, qd0)
    pots = [rng.normal(size=(4,) + tuple(d.dims)) for d in doms]
    pt = [torch.from_numpy(p).to("cuda", torch.float32) for p in pots]
    nxt = [torch.full((4,) + tuple(d.dims), float("nan"), device="cuda") for d in doms]
    e_ext = 0.7
    osc.step(pt, e_ext, nxt)
    q1, qd1, phi, psi = osc.state()
    worst = 0.0
    o = 0
    for n, (d, k) in enumerate(zip(doms, K)):
        got_s = nxt[n].double().cpu().numpy().reshape(4, -1)
        if k == 0:
            assert np.all(got_s == 0)
            continue
        P32 = pt[n].double().cpu().numpy().reshape(4, -1)
        B32 = bt[n].double().cpu().numpy().reshape(k, 4, -1)
        wphi, wpsi = cr.project(B32, P32, h)
        sl = slice(o, o + k)
        for g, w in ((phi[sl], wphi), (psi[sl], wpsi)):
            e = np.max(np.abs(g - w)) / np.max(np.abs(w))
            worst = max(worst, e)
            assert e < 1e-5, e
        wq, wqd = cr.advance(q0[sl], qd0[sl], wphi, wpsi, wpsi, e_ext, params[n], dt)
        assert np.allclose(q1[sl], wq, rtol=1e-5, atol=1e-6 * np.max(np.abs(wq)))
        assert np.allclose(qd1[sl], wqd, rtol=1e-5, atol=1e-6 * np.max(np.abs(wqd)))
        want_s = cr.synthesize(B32, q1[sl], qd1[sl])
        e = np.max(np.abs(got_s - want_s), axis=1) / np.max(np.abs(want_s), axis=1)
        worst = max(worst, float(e.max()))
        assert np.all(e < 1e-5), e
        o += k
    osc.close()
    plan.close()
    return worst


def test_one_step_at_ragged_sizes():
    h = 0.3
    doms = [sy.Domain((61, 64, 67), np.zeros(3)), sy.Domain((33, 40, 29), np.array([40.0, 0, 0])),
            sy.Domain((9, 9, 9), np.array([0.0, 40.0, 0]))]
    worst = _one_step_case(doms, [16, 3, 0], h=h)
    log(f"one oscillator step, 61x64x67 / 33x40x29 / no oscillators: worst rel err {worst:.1e}")


def test_one_step_over_more_domains_than_one_launch():
    doms = [sy.Domain((6, 7, 5), np.array([10.0 * i, 0, 0])) for i in range(18)]
    worst = _one_step_case(doms, [1 + (i % 3) for i in range(18)])
    log(f"one oscillator step over 18 domains: worst rel err {worst:.1e}")
