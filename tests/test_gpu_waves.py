"""Waves of target groups: a batch of systems split into units (targets of one
system with every domain of the system as a source, its own pad and a split
history) and packed into several batched plans.  Every target's potential,
from whichever wave evaluates it, equals the FP64 oracle run of its own
system; each wave runs one eager step and then graph replays, as the batched
benchmark does."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err
from synth import sources as sy
from test_gpu_batch import _small_batch, _subsystem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _units(system, precision, split_gap, kb=1):
    """Units and waves under a budget that halves the largest target groups
    and needs several waves (no single target above it)."""
    from paper_2311_15429_amd import waves as W
    dims, org, sid = system.dims, system.origins, np.asarray(system.system_id)
    single, groups = 0, 0
    for k in sorted(set(sid.tolist())):
        doms = list(np.where(sid == k)[0])
        for t in range(len(doms)):
            p = W._unit_plan(dims[doms], org[doms], system.h, system.dt, system.c, precision, [t], split_gap, kb)
            single = max(single, p.workspace_bytes)
            p.close()
    big = W.plan_units(dims, org, sid, system.h, system.dt, system.c, precision, budget=1 << 60, split_gap=split_gap,
                       lagsum_steps=kb)
    groups = max(u.workspace for u in big if len(u.targets) > 1)
    budget = max(single, int(0.75 * groups))
    units = W.plan_units(dims, org, sid, system.h, system.dt, system.c, precision, budget=budget, split_gap=split_gap,
                         lagsum_steps=kb)
    return big, units, W.pack_waves(units, budget), budget


@pytest.mark.parametrize("precision,tol,kb", [("fp64", 1e-10, 1), ("fp32", 2e-5, 1), ("fp32", 2e-5, 4)])
def test_waves_of_target_groups_match_the_oracle(precision, tol, kb):
    from paper_2311_15429_amd import waves as W
    system = _small_batch(3, 5)
    L = 24
    check = [6, 15, 24]
    S = sy.sample_sources(system, range(L + 1))
    big, units, waves, budget = _units(system, precision, split_gap=2, kb=kb)
    assert len(waves) >= 2 and len(units) > len(big)       # groups were halved
    covered = sorted(t for u in units for t in u.targets)
    assert covered == list(range(len(system.domains)))
    got = {l: [None] * len(system.domains) for l in check}
    dt = torch.float64 if precision == "fp64" else torch.float32
    for wi, wave in enumerate(waves):
        p, doms, targets = W.wave_plan(wave, system.dims, system.origins, system.h, system.dt, system.c,
                                       precision, split_gap=2, stream=torch.cuda.current_stream(), lagsum_steps=kb)
        assert p.workspace_bytes <= budget
        p.bind()
        p.set_green_kernels()
        tset = set(targets)
        outs = [torch.empty((4,) + p.dims[i], dtype=dt, device="cuda") if i in tset else None
                for i in range(p.n_dom)]
        buf = [torch.empty((4,) + p.dims[i], dtype=dt, device="cuda") for i in range(p.n_dom)]

        def src(l):
            return [torch.from_numpy(np.ascontiguousarray(S[g][l]).reshape((4,) + p.dims[i])).to("cuda", dt)
                    for i, g in enumerate(doms)]

        p.push_sources(0, src(0))
        p.retarded_step(0, outs)
        p.capture_step(buf, outs)
        for l in range(1, L + 1):
            for b, x in zip(buf, src(l)):
                b.copy_(x)
            p.launch_step(l)
            if l in check:
                for i in targets:
                    got[l][doms[i]] = outs[i].double().cpu().numpy().reshape(4, -1)
        torch.cuda.synchronize()
        log(f"wave {wi}: {len(wave.units)} units, {len(targets)} targets, workspace {p.workspace_bytes / 1e6:.1f} MB, "
            f"split rings {p.stats()['split_rings']}")
        p.close()
    worst = 0.0
    for s in sorted(set(system.system_id)):
        sub, idx = _subsystem(system, s)
        ref = oracle.potential_full(sub, [S[i] for i in idx], check)
        for l, r in zip(check, ref):
            e = rel_err([got[l][i] for i in idx], r)
            worst = max(worst, float(e.max()))
            assert np.all(e <= tol), (s, l, e)
    log(f"waves {precision}, {kb} steps per pass: {len(units)} units in {len(waves)} waves, worst rel err {worst:.2e}")
