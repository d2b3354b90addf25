"""Oracle driver -- TEST INFRASTRUCTURE ONLY (see the package docstring).

Functions:
  self_cell_c1()        C1 = int_{[-1/2,1/2]^3} d^3u/|u| by the oracle's own cubature.
  box_distance_range()  min/max distance between the grid points of two boxes.
  contrib()             ctypes call of the C direct sum (one source domain).
  potential_full()      every target point of every domain at the given steps.
  potential_points()    selected target points of one domain at one step.
  potential_at()        arbitrary points and times (no self cell).

The sum over sub-domains follows Eq. "multi domain ... convolution" (the
4-potential is the sum of every sub-domain's contribution).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liboracle_direct.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.rpo_contrib.restype = ctypes.c_int
    lib.rpo_contrib.argtypes = [ctypes.c_int, dp, lp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                dp, ctypes.c_double, dp, ctypes.c_long, ctypes.c_long, dp,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                ctypes.c_double, dp]
    lib.rpo_threads.restype = ctypes.c_int
    lib.rpo_threads.argtypes = [ctypes.c_int]
    _LIB = lib
    return lib


def threads(n=0):
    """Threads of the direct sum: n >= 1 sets the count; returns the count in effect."""
    return int(load_library().rpo_threads(int(n)))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------
# Self-cell constant
# ----------------------------------------------------------------------------

def self_cell_c1(n: int = 48) -> float:
    """C1 = int over the unit cube centred at 0 of 1/|u|.

    By the cube's 48-fold symmetry it is 48 times the integral over
    0 <= z <= y <= x <= 1/2; with y = x v, z = x v w the x integral gives 1/8 and
    C1 = 6 int_0^1 int_0^1 v / sqrt(1 + v^2 + v^2 w^2) dw dv, whose integrand is
    analytic on the square, so tensor Gauss-Legendre converges exponentially.
    """
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    V, W = np.meshgrid(u, u, indexing="ij")
    f = V / np.sqrt(1.0 + V * V + V * V * W * W)
    return float(6.0 * np.einsum("i,j,ij->", wu, wu, f))


# ----------------------------------------------------------------------------
# Geometry (the oracle's own; the library plans independently)
# ----------------------------------------------------------------------------

def box_distance_range(dom_t, dom_s, h):
    """Smallest and largest |r - r'| over target points r of dom_t and source
    points r' of dom_s, by brute force over the per-axis displacement values."""
    mn2 = mx2 = 0.0
    for a in range(3):
        d = np.arange(-(dom_s.dims[a] - 1), dom_t.dims[a])
        disp = (dom_t.origin[a] - dom_s.origin[a]) + h * d
        mn2 += float(np.min(np.abs(disp))) ** 2
        mx2 += float(np.max(np.abs(disp))) ** 2
    return math.sqrt(mn2), math.sqrt(mx2)


def needed_sample_range(t, rmin, rmax, dt, c, self_cell=False):
    """Sample indices [j0, j1] (j0 >= 1) that the interpolant can touch at time t
    for distances in [rmin, rmax]; (1, 0) if only S(0) is touched."""
    if math.isfinite(c):
        lo = math.floor((t - rmax / c) / dt) - 1
        hi = math.ceil((t - rmin / c) / dt) + 1
    else:
        lo = math.floor(t / dt) - 1
        hi = math.ceil(t / dt) + 1
    if self_cell:
        lstep = int(round(t / dt))
        lo = min(lo, lstep - 1)
        hi = max(hi, lstep)
    lo = max(lo, 1)
    return lo, hi


# ----------------------------------------------------------------------------
# Direct sums
# ----------------------------------------------------------------------------

def contrib(pts, self_idx, dom_s, h, samples, j0, j1, s0, t, dt, c, dynamic, c1, out):
    """Accumulate into out[n_pts][4] the contribution of source domain dom_s."""
    lib = load_library()
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n_pts = pts.shape[0]
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int64)
        sp = self_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
    else:
        sp = None
    if samples is None or j1 < j0:
        samples = np.zeros((1, 4, dom_s.n_points))
        j0, j1 = 1, 0
    samples = np.ascontiguousarray(samples, dtype=np.float64)
    s0 = np.ascontiguousarray(s0, dtype=np.float64)
    origin = np.ascontiguousarray(dom_s.origin, dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == (n_pts, 4)
    nx, ny, nz = (int(v) for v in dom_s.dims)
    rc = lib.rpo_contrib(n_pts, _dp(pts), sp, nx, ny, nz, _dp(origin), float(h),
                         _dp(samples), int(j0), int(j1), _dp(s0), float(t), float(dt),
                         float(c), int(bool(dynamic)), float(c1), _dp(out))
    if rc != 0:
        raise RuntimeError(f"oracle rpo_contrib failed with code {rc}")
    return out


def _grid_points(dom, h):
    nx, ny, nz = dom.dims
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return dom.origin[None, :] + h * pts


def _same_system(system, a, b):
    sid = system.system_id
    return sid is None or sid[a] == sid[b]


def potential_full(system, samples, steps, dynamic=False, c1=None):
    """Potential at every grid point of every domain.

    samples: list over domains of [n_samples][4][N] arrays holding S(j dt) for
    j = 0 .. n_samples-1.  Returns P[len(steps)] -> list over domains of [4][N].
    """
    if c1 is None:
        c1 = self_cell_c1()
    h, dt, c = system.h, system.dt, system.c
    result = []
    for l in steps:
        t = l * dt
        per_dom = []
        for s, dom_t in enumerate(system.domains):
            pts = _grid_points(dom_t, h)
            out = np.zeros((len(pts), 4))
            for n, dom_s in enumerate(system.domains):
                if not _same_system(system, s, n):
                    continue
                hist = samples[n]
                self_idx = np.arange(len(pts)) if n == s else None
                contrib(pts, self_idx, dom_s, h, hist[1:], 1, hist.shape[0] - 1,
                        hist[0], t, dt, c, dynamic, c1, out)
            per_dom.append(np.ascontiguousarray(out.T))
        result.append(per_dom)
    return result


def potential_points(system, s, point_idx, l, sample_fn, dynamic=False, c1=None):
    """Potential at grid points `point_idx` of target domain s at step l.

    sample_fn(n, j0, j1) -> [j1-j0+1][4][N] samples of source domain n for
    j0..j1 (j0 >= 0).  Returns [len(point_idx)][4].
    """
    if c1 is None:
        c1 = self_cell_c1()
    h, dt, c = system.h, system.dt, system.c
    t = l * dt
    dom_t = system.domains[s]
    point_idx = np.asarray(point_idx, dtype=np.int64)
    pts = _grid_points(dom_t, h)[point_idx]
    out = np.zeros((len(pts), 4))
    for n, dom_s in enumerate(system.domains):
        if not _same_system(system, s, n):
            continue
        rmin, rmax = box_distance_range(dom_t, dom_s, h)
        j0, j1 = needed_sample_range(t, rmin, rmax, dt, c, self_cell=(n == s))
        s0 = sample_fn(n, 0, 0)[0]
        hist = sample_fn(n, j0, j1) if j1 >= j0 else None
        contrib(pts, point_idx if n == s else None, dom_s, h, hist, j0, j1, s0,
                t, dt, c, dynamic, c1, out)
    return out


def potential_at(system, pts, t, sample_fn, dynamic=False, sources=None):
    """Potential at arbitrary points `pts` [n][3] and time t, none of which may
    coincide with a source grid point.  Returns [n][4]."""
    h, dt, c = system.h, system.dt, system.c
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.zeros((len(pts), 4))
    for n, dom_s in enumerate(system.domains):
        if sources is not None and n not in sources:
            continue
        lo = dom_s.origin
        hi = dom_s.origin + h * (np.array(dom_s.dims) - 1)
        near = np.clip(pts, lo, hi)
        rmin = float(np.min(np.linalg.norm(pts - near, axis=1)))
        far = np.maximum(np.abs(pts - lo), np.abs(pts - hi))
        rmax = float(np.max(np.linalg.norm(far, axis=1)))
        j0, j1 = needed_sample_range(t, rmin, rmax, dt, c)
        s0 = sample_fn(n, 0, 0)[0]
        hist = sample_fn(n, j0, j1) if j1 >= j0 else None
        contrib(pts, None, dom_s, h, hist, j0, j1, s0, t, dt, c, dynamic, 0.0, out)
    return out
