"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign, index or lag, a transposed operand, a wrong self cell) fails at
least one of them:

* self-cell constant vs its closed form;
* Hartree limit (c -> infinity) vs the Gaussian-charge potential q erf(r/s)/r,
  far field to spectral accuracy and self-domain O(h^2) convergence;
* causality: the dynamic part is exactly zero before light arrives;
* the far field of an oscillating +/- pair vs the retarded dipole potentials,
  and its broadside E field vs the paper's Hertzian-dipole formula
  (Sec. "Results", Eq. "electric field inf dipole");
* the Lorenz gauge condition (Appendix B, Eq. "lorenz gauge fixing") on the
  oracle's phi and A, converging as dt shrinks;
* brute force of the paper's discrete lag-sum form (Eq. "retardation
  space-time sampled lorentz four vector potential" with the sampled Green's
  function of Eq. "retardation space-time sampled green interpolation") on
  tiny inputs, a different formula from the oracle's interpolated direct sum;
* step response -> static Coulomb sum; static + dynamic split; exact symmetries;
  the self pair's sampled kernel is even, so its padded DFT is real.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle_helpers import Charge, System, array_sample_fn, centred, grid_points, sample_fn_for

C_AU = 137.036


# ---------------------------------------------------------------------------
def test_self_cell_constant_closed_form():
    # int_{[-1/2,1/2]^3} d^3u/|u| = 3 ln((sqrt3+1)/(sqrt3-1)) - pi/2 = 3 ln(2+sqrt3) - pi/2
    closed = 3.0 * math.log((math.sqrt(3) + 1) / (math.sqrt(3) - 1)) - math.pi / 2
    assert abs(oracle.self_cell_c1() - closed) < 1e-13
    assert abs(closed - 2.380077363979554) < 1e-14


# ---------------------------------------------------------------------------
def test_hartree_limit_far_domain():
    """c = inf, a static Gaussian charge >= 6 s inside its box: the potential in
    another domain is q erf(r/s)/r up to the grid's spectral error
    ~ exp(-(pi s/h)^2)."""
    h, s, q = 0.5, 1.0, 0.7
    centre = np.array([0.1, -0.2, 0.15])
    A = centred((0, 0, 0), 27, h)
    A.charges.append(Charge("single", s, centre, None, ("const", q)))
    B = centred((20.0, 5.0, -3.0), 4, h)
    sy = System(h, 0.02, math.inf, [A, B])
    P = oracle.potential_points(sy, 1, np.arange(64), 0, sample_fn_for(sy))
    r = np.linalg.norm(grid_points(B, h) - centre, axis=1)
    exact = q * erf(r / s) / r
    assert np.max(np.abs(P[:, 0] - exact)) / np.max(np.abs(exact)) < 1e-9
    assert np.all(P[:, 1:] == 0.0)


def _near_field_error(h, s=1.0, q=0.7, side=12.0):
    n = int(round(side / h)) + 1
    A = centred((0, 0, 0), n, h)
    A.charges.append(Charge("single", s, np.zeros(3), None, ("const", q)))
    sy = System(h, 0.02, math.inf, [A])
    pts = grid_points(A, h)
    # points on the +x axis at multiples of 0.4 bohr, common to both grids
    sel = [i for i, p in enumerate(pts)
           if abs(p[1]) < 1e-9 and abs(p[2]) < 1e-9 and -1e-9 < p[0] < 2.5
           and abs(p[0] / 0.4 - round(p[0] / 0.4)) < 1e-6]
    P = oracle.potential_points(sy, 0, sel, 0, sample_fn_for(sy))
    r = np.linalg.norm(pts[sel], axis=1)
    exact = np.where(r > 0, q * erf(r / s) / np.where(r > 0, r, 1.0), 2 * q / (s * math.sqrt(math.pi)))
    self_term = h * h * oracle.self_cell_c1() * q * (math.pi * s * s) ** -1.5
    return np.max(np.abs(P[:, 0] - exact)), self_term


def test_hartree_limit_self_domain_converges_h2():
    e1, self1 = _near_field_error(0.4)
    e2, _ = _near_field_error(0.2)
    assert 3.2 < e1 / e2 < 4.8          # O(h^2)
    assert e1 < 0.3 * self1             # the self cell is present and of the right size


# ---------------------------------------------------------------------------
def test_causality_exact_zero_before_arrival():
    h, dt = 0.5, 0.02
    A = centred((0, 0, 0), 8, h)
    A.charges.append(Charge("pair", 0.9, np.array([0.5, 0.2, -0.3]), np.array([-0.6, -0.1, 0.4]),
                            ("cos", 0.8, 0.4, 1.1)))
    B = centred((25.0, 3.0, 0.0), 6, h)       # no sources of its own
    sy = System(h, dt, C_AU, [A, B])
    fn = sample_fn_for(sy)
    rmin, _ = oracle.box_distance_range(B, A, h)
    l_last_zero = int(math.floor(rmin / (C_AU * dt)))
    for l in (0, 1, l_last_zero):
        assert l * dt <= rmin / C_AU
        P = oracle.potential_points(sy, 1, np.arange(B.n_points), l, fn, dynamic=True)
        assert np.all(P == 0.0), l
    P = oracle.potential_points(sy, 1, np.arange(B.n_points), l_last_zero + 1, fn, dynamic=True)
    assert np.max(np.abs(P)) > 0.0
    # in the source's own domain the dynamic part is nonzero from step 1
    P = oracle.potential_points(sy, 0, np.arange(A.n_points), 1, fn, dynamic=True)
    assert np.max(np.abs(P)) > 0.0


# ---------------------------------------------------------------------------
def _dipole_system(dt):
    h, w, q0, sep, s = 0.25, 0.5, 1.0, 2.0, 0.5
    A = centred((0, 0, 0), 41, h)
    A.charges.append(Charge("pair", s, np.array([0, 0, sep / 2]), np.array([0, 0, -sep / 2]),
                            ("cos", q0, w, -math.pi / 2)))      # q(t) = q0 sin(w t)
    return System(h, dt, C_AU, [A]), w, q0 * sep


def _dipole_errors(dt, r=200.0):
    sy, w, p0 = _dipole_system(dt)
    fn = sample_fn_for(sy)
    c = C_AU
    ts = r / c + 0.2 + np.arange(12) * (2 * math.pi / w) / 12
    errs = []
    for d in (np.array([0, 0, 1.0]), np.array([1, 1, 1.0]) / math.sqrt(3), np.array([0.3, -0.5, 0.81])):
        d = d / np.linalg.norm(d)
        got, ref = [], []
        for t in ts:
            P = oracle.potential_at(sy, (r * d)[None, :], t, fn)[0]
            tr = t - r / c
            p, pd = p0 * math.sin(w * tr), p0 * w * math.cos(w * tr)
            # Gaussian a.u.: phi = n.[p/r^2 + pdot/(c r)],  A = pdot/(c r)  (p along z)
            ref.append([d[2] * (p / r ** 2 + pd / (c * r)), 0.0, 0.0, pd / (c * r)])
            got.append(P)
        got, ref = np.array(got), np.array(ref)
        errs.append(np.max(np.abs(got[:, 0] - ref[:, 0])) / np.max(np.abs(ref[:, 0])))
        errs.append(np.max(np.abs(got[:, 3] - ref[:, 3])) / np.max(np.abs(ref[:, 3])))
        assert np.max(np.abs(got[:, 1:3])) < 1e-12 * np.max(np.abs(ref[:, 3]))
    return max(errs)


def test_oscillating_dipole_far_field():
    """Far field of a +/- pair q(t) = q0 sin(w t) at +-1 bohr on z, at r = 200:
    error O((d/r)^2) + linear-interpolation error ~ (w dt)^2 r/d."""
    e_fine = _dipole_errors(0.005)
    e_coarse = _dipole_errors(0.02)
    assert e_fine < 1e-4
    assert e_coarse / e_fine > 8.0          # interpolation error ~ dt^2


def test_broadside_field_matches_hertzian_dipole_formula():
    """E_z = -d_z phi - (1/c) d_t A_z at a broadside point vs the paper's
    Hertzian-dipole field Re[p e^{-i w (t - t_r)} (w^2/(c^2 d) + i w/(c d^2) - 1/d^3)]
    (Gaussian a.u., charge dipole p = q0 sep sin(w t) = Re[i q0 sep e^{-i w t}])."""
    dt = 0.005
    sy, w, p0 = _dipole_system(dt)
    fn = sample_fn_for(sy)
    c, r = C_AU, 200.0
    x0 = np.array([r, 0.0, 0.0])
    dl = 0.5
    got, ref = [], []
    for t in r / c + 0.2 + np.arange(8) * (2 * math.pi / w) / 8:
        Pz = oracle.potential_at(sy, np.array([x0 + [0, 0, dl], x0 - [0, 0, dl]]), t, fn)
        Pt = oracle.potential_at(sy, np.array([x0]), t + dt, fn)[0]
        Pm = oracle.potential_at(sy, np.array([x0]), t - dt, fn)[0]
        got.append(-(Pz[0, 0] - Pz[1, 0]) / (2 * dl) - (Pt[3] - Pm[3]) / (2 * dt) / c)
        phat = 1j * p0
        ref.append((phat * np.exp(-1j * w * (t - r / c))
                    * (w ** 2 / (c ** 2 * r) + 1j * w / (c * r ** 2) - 1 / r ** 3)).real)
    got, ref = np.array(got), np.array(ref)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-3


# ---------------------------------------------------------------------------
def _lorenz_residual(dt, h=0.25):
    A = centred((0, 0, 0), 41, h)
    A.charges.append(Charge("pair", 0.6, np.array([0.5, -0.3, 1.0]), np.array([-0.7, 0.4, -0.8]),
                            ("cos", 0.8, 0.5, 0.3)))
    c = C_AU
    sy = System(h, dt, c, [A])
    fn = sample_fn_for(sy)
    rng = np.random.default_rng(5)
    pts = rng.normal(size=(6, 3))
    pts = pts / np.linalg.norm(pts, axis=1)[:, None] * rng.uniform(12, 30, size=(6, 1))
    d, dtt = 0.01, 1e-4
    res, scale = [], []
    for t in 30 / c + 0.3 + rng.uniform(0, 12, size=5):   # every retarded time > dt
        off = []
        for a in range(3):
            e = np.zeros(3)
            e[a] = d
            off += [pts + e, pts - e]
        P = oracle.potential_at(sy, np.concatenate(off), t, fn).reshape(6, len(pts), 4)
        div_a = sum((P[2 * a][:, 1 + a] - P[2 * a + 1][:, 1 + a]) / (2 * d) for a in range(3))
        dphi = (oracle.potential_at(sy, pts, t + dtt, fn)[:, 0]
                - oracle.potential_at(sy, pts, t - dtt, fn)[:, 0]) / (2 * dtt) / c
        res.append(div_a + dphi)
        scale.append(dphi)
    return np.max(np.abs(res)) / np.max(np.abs(scale))


def test_lorenz_condition_converges():
    """div A + (1/c) d_t phi = 0 for continuity-satisfying sources; linear time
    interpolation leaves an O(dt) pointwise residual."""
    r = [_lorenz_residual(dt) for dt in (0.04, 0.02, 0.01)]
    assert r[0] < 0.08
    assert r[0] / r[1] > 1.8 and r[1] / r[2] > 1.8


# ---------------------------------------------------------------------------
def _self_kernel_cubature(m, h, dt, c, n=24):
    """int_cell T(m dt - |u|/c)/|u| d^3u over the cube of side h centred at 0,
    with T(x) = max(0, 1 - |x|/dt), in coordinates u = (x, x v, x v w) on the
    fundamental 1/48 of the cube (T is polynomial in x on the cell here)."""
    g, wg = np.polynomial.legendre.leggauss(n)
    x = 0.25 * h * (g + 1.0)
    wx = 0.25 * h * wg
    v = 0.5 * (g + 1.0)
    wv = 0.5 * wg
    X, V, W = np.meshgrid(x, v, v, indexing="ij")
    rho = np.sqrt(1.0 + V * V + V * V * W * W)
    R = X * rho
    if math.isfinite(c):
        T = np.maximum(0.0, 1.0 - np.abs(m * dt - R / c) / dt)
    else:
        T = np.ones_like(R) if m == 0 else np.zeros_like(R)
    f = X * V * T / rho
    return 48.0 * np.einsum("i,j,k,ijk->", wx, wv, wv, f)


def _lag_sum_bruteforce(domains, h, dt, c, S, L):
    """P(r_k, l dt) = sum_n [ P_n(r_k, 0) + sum_{k'} sum_{l'=1}^{l} G_{l-l'}[k,k'] dS(r_k', l') ]
    with G_m[k,k'] = h^3 T(m dt - R/c)/R and the self point's cell integral."""
    T = lambda x: max(0.0, 1.0 - abs(x) / dt)
    pts = [grid_points(d, h) for d in domains]
    w_self = [_self_kernel_cubature(m, h, dt, c) for m in range(L + 1)]
    w_static = _self_kernel_cubature(0, h, dt, math.inf)
    out = np.zeros((L + 1, len(domains), 4, max(len(p) for p in pts)))
    for s, pt in enumerate(pts):
        for k, r in enumerate(pt):
            for n, ps in enumerate(pts):
                for kp, rp in enumerate(ps):
                    R = float(np.linalg.norm(r - rp))
                    self_pt = (n == s and kp == k)
                    g_static = w_static if self_pt else h ** 3 / R
                    for l in range(L + 1):
                        acc = g_static * S[n][0, :, kp]
                        for lp in range(1, l + 1):
                            m = l - lp
                            g = w_self[m] if self_pt else h ** 3 * T(m * dt - R / c) / R
                            if g != 0.0:
                                acc = acc + g * (S[n][lp, :, kp] - S[n][0, :, kp])
                        out[l, s, :, k] += acc
    return out


def test_oracle_equals_lag_sum_bruteforce():
    h, dt, c, L = 0.5, 0.05, 10.0, 12
    rng = np.random.default_rng(11)
    doms = [centred((0, 0, 0), 2, h), centred((1.9, 0.7, -0.4), 2, h)]
    sy = System(h, dt, c, doms)
    S = [rng.normal(size=(L + 1, 4, d.n_points)) for d in doms]
    ref = _lag_sum_bruteforce(doms, h, dt, c, S, L)
    got = oracle.potential_full(sy, S, range(L + 1))
    for l in range(L + 1):
        for s in range(2):
            np.testing.assert_allclose(got[l][s], ref[l, s], rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    # the history really is retarded: early steps differ from the instantaneous sum
    inst = oracle.potential_full(System(h, dt, math.inf, doms), S, [L])
    assert np.max(np.abs(inst[0][1] - got[L][1])) > 1e-3


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c,dt", [(C_AU, 0.002), (10.0, 0.03)])
def test_self_pair_kernel_is_even_so_its_spectrum_is_real(c, dt):
    """The sampled Green's function of a domain on itself at every lag m (the
    response at step m + 1 to a unit source difference at step 1 in the centre
    point, self cell included) is even under r -> -r, so its DFT on a padded
    grid (offset r at index r mod P) is real: the FP32 path keeps only the real
    parts of the self pairs' spectra."""
    h, n, P = 0.25, 9, 20
    dom = centred((0.0, 0.0, 0.0), n, h)
    sy = System(h, dt, c, [dom])
    L = 12
    centre = (n // 2) * (n * n + n + 1)
    S = np.zeros((L + 1, 4, dom.n_points))
    S[1, 0, centre] = 1.0
    got = oracle.potential_full(sy, [S], range(2, L + 1))
    nonzero = 0
    for l, per in zip(range(2, L + 1), got):
        g = per[0][0].reshape(n, n, n)
        scale = np.max(np.abs(g))
        if scale == 0.0:
            continue
        nonzero += 1
        for axes in ((0,), (1,), (2,), (0, 1, 2)):
            np.testing.assert_allclose(g, np.flip(g, axis=axes), rtol=0, atol=1e-14 * scale)
        pad = np.zeros((P, P, P))
        idx = (np.arange(n) - n // 2) % P
        pad[np.ix_(idx, idx, idx)] = g
        spec = np.fft.fftn(pad)
        assert np.max(np.abs(spec.imag)) <= 1e-13 * np.max(np.abs(spec.real)), l
        # a kernel shifted off the centre (a cross pair) is not even
        shifted = np.fft.fftn(np.roll(pad, 1, axis=0))
        assert np.max(np.abs(shifted.imag)) > 1e-3 * np.max(np.abs(shifted.real))
    assert nonzero >= 3


# ---------------------------------------------------------------------------
def test_step_response_reaches_static_coulomb_sum():
    """Sources jump to S1 at step 1 and hold: once every retarded time exceeds dt
    the potential is the instantaneous Coulomb sum of S1."""
    h, dt = 0.5, 0.02
    mk = lambda prof_a, prof_b: [
        _with(centred((0, 0, 0), 6, h), Charge("single", 0.8, np.array([0.1, 0.2, -0.1]), None, prof_a)),
        _with(centred((8.0, -2.0, 1.0), 6, h), Charge("single", 1.1, np.array([8.2, -2.1, 1.0]), None, prof_b))]
    sy = System(h, dt, C_AU, mk(("step", 0.3, -0.9), ("step", -0.5, 0.4)))
    st = System(h, dt, math.inf, mk(("const", -0.9), ("const", 0.4)))
    _, rmax = oracle.box_distance_range(sy.domains[0], sy.domains[1], h)
    l = int(math.ceil(rmax / (C_AU * dt))) + 2
    fa, fb = sample_fn_for(sy), sample_fn_for(st)
    for s in range(2):
        idx = np.arange(sy.domains[s].n_points)
        got = oracle.potential_points(sy, s, idx, l, fa)
        ref = oracle.potential_points(st, s, idx, 0, fb)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


def _with(dom, ch):
    dom.charges.append(ch)
    return dom


# ---------------------------------------------------------------------------
def _random_pair_system(c=C_AU, shift=(0.0, 0.0, 0.0), swap=False, seed=3):
    rng = np.random.default_rng(seed)
    h, dt = 0.5, 0.02
    shift = np.asarray(shift)
    doms = [centred(np.array([0, 0, 0.0]) + shift, 5, h), centred(np.array([9.0, 1.0, -2.0]) + shift, 4, h)]
    for d in doms:
        lo = d.origin
        hi = d.origin + h * (np.array(d.dims) - 1)
        for _ in range(2):
            d.charges.append(Charge("pair", rng.uniform(0.8, 1.5), rng.uniform(lo, hi), rng.uniform(lo, hi),
                                    ("cos", rng.uniform(0.1, 1), rng.uniform(0.1, 0.5), rng.uniform(0, 6.28))))
    if swap:
        doms = doms[::-1]
    return System(h, dt, c, doms)


def _full(sy, steps):
    fn = sample_fn_for(sy)
    L = max(steps)
    S = [fn(n, 0, L) for n in range(len(sy.domains))]
    return oracle.potential_full(sy, S, steps), S


def test_static_plus_dynamic_split():
    sy = _random_pair_system()
    steps = [0, 3, 9]
    tot, S = _full(sy, steps)
    dyn = oracle.potential_full(sy, S, steps, dynamic=True)
    for i in range(len(steps)):
        for s in range(2):
            scale = np.max(np.abs(tot[i][s]))
            np.testing.assert_allclose(tot[i][s] - tot[0][s], dyn[i][s], rtol=0, atol=1e-13 * scale)
    assert all(np.all(d == 0.0) for d in dyn[0])


def test_translation_and_permutation_invariance():
    steps = [2, 7]
    base, _ = _full(_random_pair_system(), steps)
    moved, _ = _full(_random_pair_system(shift=(13.3, -7.1, 2.2)), steps)
    swapped, _ = _full(_random_pair_system(swap=True), steps)
    for i in range(len(steps)):
        for s in range(2):
            scale = np.max(np.abs(base[i][s]))
            np.testing.assert_allclose(moved[i][s], base[i][s], rtol=0, atol=1e-12 * scale)
            np.testing.assert_allclose(swapped[i][1 - s], base[i][s], rtol=0, atol=1e-14 * scale)


def test_superposition():
    sy = _random_pair_system()
    rng = np.random.default_rng(7)
    L = 8
    Sa = [rng.normal(size=(L + 1, 4, d.n_points)) for d in sy.domains]
    Sb = [rng.normal(size=(L + 1, 4, d.n_points)) for d in sy.domains]
    Pa = oracle.potential_full(sy, Sa, [L])
    Pb = oracle.potential_full(sy, Sb, [L])
    Pab = oracle.potential_full(sy, [a + b for a, b in zip(Sa, Sb)], [L])
    for s in range(2):
        scale = np.max(np.abs(Pab[0][s]))
        np.testing.assert_allclose(Pab[0][s], Pa[0][s] + Pb[0][s], rtol=0, atol=1e-13 * scale)
