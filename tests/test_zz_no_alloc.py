"""A plan bound to the library's fixed device array (rp_bind_workspace_static,
which allocates nothing) gives the results of the same plan bound to a
caller-allocated workspace (rp_bind_workspace): two plans in a row on the
array, the second smaller, each checked against its twin on a workspace and
against the FP64 oracle (1e-10)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STEPS = 20                  # past the deepest lag (15) of the two-domain case
CHECK = [1, 9, 17, 20]


def _system(n):
    """The FP64 two-domain case (h = 0.5, centres 30 bohr apart on x, dt =
    0.02) with n^3 points per domain around the same centres."""
    s = sy.config1(1)
    for d in s.domains:
        centre = d.origin + 0.5 * 15 * s.h
        d.dims = (n, n, n)
        d.origin = centre - 0.5 * (n - 1) * s.h
    return s


def _start(system, static):
    from paper_2311_15429_amd import plan_for_system
    plan = plan_for_system(system, "fp64", stream=torch.cuda.current_stream())
    if static:
        plan.bind_static()
    else:
        plan.bind()
    plan.set_green_kernels()
    return plan


def _steps(plan, S, steps):
    outs = [torch.empty((4,) + d, dtype=torch.float64, device="cuda") for d in plan.dims]
    got = {}
    for l in steps:
        plan.push_sources(l, [torch.from_numpy(np.ascontiguousarray(S[n][l]).reshape((4,) + plan.dims[n]))
                              .to("cuda") for n in range(plan.n_dom)])
        plan.retarded_step(l, outs)
        if l in CHECK:
            got[l] = [o.cpu().numpy().reshape(4, -1) for o in outs]
    torch.cuda.synchronize()
    return got


def _check(system, S, got_static, got_ws, label):
    ref = oracle.potential_full(system, S, CHECK)
    for l, r in zip(CHECK, ref):
        for a, b in zip(got_static[l], got_ws[l]):
            assert np.array_equal(a, b), (label, l)
        e = rel_err(got_static[l], r)
        log(f"  [{label}] step {l}: rel err vs oracle " + " ".join(f"{x:.2e}" for x in e))
        assert np.all(e <= 1e-10), (label, l, e)


def test_fixed_array_bind_matches_caller_workspace():
    from paper_2311_15429_amd import RpotError
    big, small = _system(16), _system(8)
    S_big = sy.sample_sources(big, range(STEPS + 1))
    S_small = sy.sample_sources(small, range(STEPS + 1))

    # first call: the 2 x 16^3 plan (52 MiB of the 64 MiB array)
    a = _start(big, static=True)
    assert a.workspace_bytes > 48 << 20
    got_a = _steps(a, S_big, range(0, 10))
    ref_a = _start(big, static=False)
    ws_a = _steps(ref_a, S_big, range(0, STEPS + 1))

    # second call, smaller: it takes the array over from the first plan
    b = _start(small, static=True)
    with pytest.raises(RpotError) as ei:
        _steps(a, S_big, [10])
    assert ei.value.code == 4
    got_b = _steps(b, S_small, range(0, STEPS + 1))
    ref_b = _start(small, static=False)
    ws_b = _steps(ref_b, S_small, range(0, STEPS + 1))
    _check(small, S_small, got_b, ws_b, "2 x 8^3 on the array")

    # the first plan bound again restarts its sequence on the array
    a.bind_static()
    a.set_green_kernels()
    got_a = _steps(a, S_big, range(0, STEPS + 1))
    _check(big, S_big, got_a, ws_a, "2 x 16^3 on the array, bound again")
    for p in (a, b, ref_a, ref_b):
        p.close()


def test_fixed_array_rejects_a_plan_that_does_not_fit():
    from paper_2311_15429_amd import RpotError, plan_for_system
    p = plan_for_system(_system(24), "fp64", stream=torch.cuda.current_stream())
    assert p.workspace_bytes > 64 << 20
    with pytest.raises(RpotError) as ei:
        p.bind_static()
    assert ei.value.code == 3 and "fixed array" in str(ei.value)
    with pytest.raises(RpotError):          # nothing was bound
        p.set_green_kernels()
    p.close()
