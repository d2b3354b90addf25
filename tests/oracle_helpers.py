"""Small builders shared by the oracle pin tests (inputs only)."""
from __future__ import annotations

import math

import numpy as np

from synth.sources import Charge, Domain, System, spatial_factors, time_factors, grid_points


def centred(centre, n, h):
    centre = np.asarray(centre, dtype=np.float64)
    if np.isscalar(n):
        n = (n, n, n)
    return Domain(tuple(int(v) for v in n), centre - 0.5 * (np.array(n) - 1) * h)


def sample_fn_for(system: System):
    """sample_fn(n, j0, j1) -> [j1-j0+1][4][N] from the separable sources."""
    B = [spatial_factors(d, system.h, system.c) for d in system.domains]

    def fn(n, j0, j1):
        A = time_factors(system.domains[n], system.dt, np.arange(j0, j1 + 1))
        nt = B[n].shape[0]
        if nt == 0:
            return np.zeros((j1 - j0 + 1, 4, system.domains[n].n_points))
        return (A @ B[n].reshape(nt, -1)).reshape(j1 - j0 + 1, 4, -1)

    return fn


def array_sample_fn(samples):
    """sample_fn over explicit sample arrays samples[n][j][4][N] (j from 0)."""
    def fn(n, j0, j1):
        return samples[n][j0:j1 + 1]
    return fn


__all__ = ["centred", "sample_fn_for", "array_sample_fn", "Charge", "Domain", "System",
           "grid_points", "math"]
