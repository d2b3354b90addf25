"""Judge by sample: the far pairs of non-audit sources are judged by the
direct sum at 64 sample points from a real-space history, and fall back into
slots of their own.  Sample fields against the FP64 oracle; a non-audit pair
falling back and the whole output then matching the oracle at every later
step (FP32 and I16 rings); rotation coverage, refused fallbacks when the
slots are full, re-admission freeing the slots."""
import numpy as np
import pytest

import oracle
from oracle import surrogate_ref as sr
from gpu_helpers import GpuSourceGen, log, rel_err
from synth import sources as sy
from test_gpu_surrogate import FAR, N_LAGS, far_system, pair_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _sample_idx(N):
    """Linear grid indices of the 64 sample points (16 a_x + 4 a_y + a_z)."""
    ax = [(a * (n - 1) + 1) // 3 for n in N for a in range(4)]
    ix, iy, iz = ax[0:4], ax[4:8], ax[8:12]
    return np.array([(ix[p >> 4] * N[1] + iy[(p >> 2) & 3]) * N[2] + iz[p & 3] for p in range(64)])


def _all_arrived(p, pairs):
    """A step at which every far pair's field has arrived (past each window's
    first lag by a few steps)."""
    return max(p.info(int(t), int(n))[0] for t, n in zip(pairs["target"], pairs["source"])) + 4


def _plan(system, audit, per_judge, slots, precision="fp32", steps=1):
    from paper_2311_15429_amd import plan_for_system
    p = plan_for_system(system, precision, stream=torch.cuda.current_stream())
    if steps > 1:
        p.set_tuning("lagsum_steps", steps)
    p.surrogate_configure(FAR, n_lags=N_LAGS, audit=audit)
    p.surrogate_sample(per_judge, slots)
    p.bind()
    p.set_green_kernels()
    return p


def test_sample_fields_match_the_oracle_direct_sum():
    system = far_system(11)
    L = 44
    S = sy.sample_sources(system, range(L + 1))
    p = _plan(system, audit=[2], per_judge=0, slots=0)
    gen = GpuSourceGen(system, torch.float32)
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(L + 1):
        p.push_sources(l, gen.step(l))
        p.retarded_step(l, outs)
    pairs = p.surrogate_pairs()
    nf = len(pairs["target"])
    got = p.surrogate_sample_fields(np.arange(nf), torch.empty((nf, 64, 4), device="cuda")).double().cpu().numpy()
    worst = 0.0
    for f in range(nf):
        s, n = int(pairs["target"][f]), int(pairs["source"][f])
        F = pair_field(system, S, s, n, L)[:, _sample_idx(system.domains[s].dims)].T      # [64][4]
        scale = np.max(np.abs(F))
        assert scale > 0, (s, n)
        e = np.max(np.abs(got[f] - F)) / scale
        worst = max(worst, e)
        assert e <= 1e-5, (f, s, n, e)
    log(f"sample fields: {nf} far pairs (audited and not) at 64 points, worst rel err {worst:.2e}")
    p.close()


@pytest.mark.parametrize("precision,tol,steps", [("fp32", 2e-5, 1), ("fp32_ring_i16", 1e-4, 1), ("fp32", 2e-5, 4),
                                                ("fp32_ring_i16", 1e-4, 8)])
def test_non_audit_pairs_fall_back_into_slots_and_match_the_oracle(precision, tol, steps):
    """Multipole terms judged with a tiny tolerance: every far pair fails,
    audited ones into the plain lag sum, the others into fallback slots
    (refilled from the real-space history, Green spectra computed then).  From
    the next step on the whole output is the plain method's.  With blocked
    lag-sum steps (4 or 8 per pass) the judge runs after the last step of a
    block, the blocked schedules are rebuilt with the fallen-back pairs, and
    the slots add their pairs step by step into the block's accumulators."""
    system = far_system(12)
    p = _plan(system, audit=[2], per_judge=0, slots=32, precision=precision, steps=steps)
    p.surrogate_multipole(True)
    pairs = p.surrogate_pairs()
    Lj = _all_arrived(p, pairs)
    Lj += (-Lj) % steps                   # a block's last step (blocks start at steps 1, 1 + kb, ...)
    L = Lj + 14
    S = sy.sample_sources(system, range(L + 1))
    n_far_nonaudit = int((~pairs["audited"]).sum())
    assert n_far_nonaudit > 0 and pairs["audited"].any()
    gen = GpuSourceGen(system, torch.float32)
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    got = {}
    bytes0 = p.stats()["lagsum_bytes"]
    for l in range(L + 1):
        p.push_sources(l, gen.step(l))
        p.retarded_step(l, outs)
        if steps > 1 and l == Lj - 1:
            with pytest.raises(Exception, match="last step of a block"):
                p.surrogate_judge(outs, 1e-9)
        if l == Lj:
            nf, worst = p.surrogate_judge(outs, 1e-9)
            st = p.surrogate_judge_stats()
            assert nf == len(pairs["target"]) and worst > 1
            assert st["sampled"] == n_far_nonaudit and st["refused"] == 0
            assert st["slots_used"] == n_far_nonaudit
            assert p.surrogate_pairs()["fallen_back"].all()
            assert p.stats()["lagsum_bytes"] > bytes0
        if l > Lj:
            got[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    ref = oracle.potential_full(system, S, sorted(got))
    worst = 0.0
    for (l, g), r in zip(sorted(got.items()), ref):
        e = rel_err(g, r)
        worst = max(worst, float(e.max()))
        assert np.all(e <= tol), (l, e)
    log(f"{precision}, {steps} steps per pass: {n_far_nonaudit} non-audit pairs in slots; steps {Lj + 1}..{L} "
        f"vs oracle {worst:.2e}")
    p.close()


def test_rotation_refusal_and_readmission():
    """Three sampled pairs per call and two slots: the rotation reaches every
    non-audit pair within ceil(n / 3) calls; fallbacks beyond the slots are
    refused; re-admission frees the slots and the output returns to the
    surrogate-only plan's."""
    system = far_system(13)
    p = _plan(system, audit=[2], per_judge=3, slots=2)
    p.surrogate_multipole(True)
    pairs = p.surrogate_pairs()
    L = _all_arrived(p, pairs)
    sampled = [f for f in range(len(pairs["target"])) if not pairs["audited"][f]]
    gen = GpuSourceGen(system, torch.float32)
    outs = [torch.empty((4,) + d, dtype=torch.float32, device="cuda") for d in p.dims]
    for l in range(L + 1):
        p.push_sources(l, gen.step(l))
        p.retarded_step(l, outs)
    seen, refused = [], 0
    calls = -(-len(sampled) // 3)
    for c in range(calls):
        seen.append(p.surrogate_judge_stats()["next_pair"])
        p.surrogate_judge(outs, 1e-9)
        st = p.surrogate_judge_stats()
        assert st["sampled"] == min(3, len(sampled))
        refused += st["refused"]
    assert seen[0] == sampled[0]
    assert p.surrogate_judge_stats()["slots_used"] == 2
    assert refused == len(sampled) - 2
    fb = p.surrogate_pairs()["fallen_back"]
    assert int(fb[sampled].sum()) == 2
    # every non-audit pair was judged: the cursor went round once
    assert p.surrogate_judge_stats()["next_pair"] == sampled[(calls * 3) % len(sampled)]
    # re-admission: a loose tolerance returns the slot pairs
    p.surrogate_readmit(1e30)
    back = 0
    for c in range(calls):
        p.surrogate_judge(outs, 1e3)
        back += p.last_readmitted
    assert p.surrogate_judge_stats()["slots_used"] == 0
    assert not p.surrogate_pairs()["fallen_back"][sampled].any()
    log(f"rotation: {len(sampled)} sampled pairs in {calls} calls, {refused} refused, {back} re-admitted")
    p.close()
