"""The multi-domain split is exact (Sec. II-III): two sub-domains computed as
two domains give, on their points, the same potentials as one domain that
encloses both and holds their sources, zero elsewhere.  Both runs go through
the C-ABI; the two discrete sums are the same sum, and both are also checked
against the FP64 oracle of the two-domain system."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, run_gpu
from synth import sources as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _scatter(system, encl, blocks, S):
    """Sources of the enclosing domain: [L+1][4][N] with each sub-domain's
    samples in its block and zero elsewhere."""
    dims = encl.domains[0].dims
    L1 = S[0].shape[0]
    big = np.zeros((L1, 4) + tuple(dims))
    for n, dm in enumerate(system.domains):
        big[(slice(None), slice(None)) + blocks[n]] = S[n].reshape((L1, 4) + tuple(dm.dims))
    return [big.reshape(L1, 4, -1)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_two_domains_equal_one_enclosing_domain(precision, tol):
    system = sy.wire_pair(W=8, L=24, d=40, h=0.5, dt=0.005, n_pairs=2, seed=3)
    encl, blocks = sy.enclosing_domain(system)
    L = 70
    steps = [20, 45, L]
    S = sy.sample_sources(system, range(L + 1))
    multi = run_gpu(system, precision, S, collect=steps)
    single = run_gpu(encl, precision, _scatter(system, encl, blocks, S), collect=steps)
    dims = encl.domains[0].dims
    ref = oracle.potential_full(system, S, steps)
    for i, l in enumerate(steps):
        big = single[l][0].reshape((4,) + tuple(dims))
        cut = [big[(slice(None),) + b].reshape(4, -1) for b in blocks]
        e = rel_err(multi[l], cut)
        eo_multi, eo_single = rel_err(multi[l], ref[i]), rel_err(cut, ref[i])
        log(f"{precision} step {l}: two domains vs enclosing domain, rel diff {np.array2string(e, precision=2)}; "
            f"vs oracle {eo_multi.max():.1e} / {eo_single.max():.1e}")
        assert np.all(e <= tol), (l, e)
        assert np.all(eo_multi <= tol) and np.all(eo_single <= tol), (l, eo_multi, eo_single)
