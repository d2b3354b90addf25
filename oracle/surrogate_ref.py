"""FP64 reference of the fixed (not learned) parts of the far-pair surrogate.

Test infrastructure: only tests/, the smoke check and the bench's CPU baseline
use this module.  It shares no code with the HIP path.

The paper ends by naming a multipole approximation of far sub-domains' retarded
potentials as a further speed-up (Sec. V, conclusion).  The surrogate learns
that far coupling; what it computes besides the network is defined here from
first principles:

* moments of dS = S(t) - S(0) of a source domain about its box centre c, with
  the quadrature weight h^3 of the discrete lag sum (Sec. III): charge q,
  dipole p, second moment Q (xx yy zz xy xz yz), current monopole J and current
  first moment K_ij = sum dS_{1+i} x_j;
* the pair frame: e1 along c_target - c_source, e2 the unit part of a reference
  axis (z, or x when e1 is within 25.8 degrees of z) orthogonal to e1,
  e3 = e1 x e2;
* the network input of a pair at step l: H = moments of steps l - m for the
  lags m = m_c - n_lags/2 + j, rotated into the frame (vectors R v, tensors
  R T R^T); with g = 10 dbar / |d| and f = |d|/(c dt) - m_c the six blocks
  H, g H, f H, g f H, g^2 H, f^2 H, then g and f;
* the cubic tensor-Legendre basis P_i(x) P_j(y) P_k(z), i + j + k <= 3, and the
  least-squares coefficients of a field on the target grid in the frame
  variables u = R (r - c_target) / ell (A components taken in the frame).

Parity of the learned output itself is unpinned: it is an approximation,
judged against the plain lag sum and the direct sum at sampled points.
"""
from __future__ import annotations

import math

import numpy as np

DEGREES = [(i, j, k) for i in range(4) for j in range(4) for k in range(4) if i + j + k <= 3]
N_FEAT = 22
N_GEO = 2
N_BLOCKS = 6


def grid_points(dom, h):
    axes = [dom.origin[a] + h * np.arange(dom.dims[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def box_centre(dom, h):
    return np.asarray(dom.origin, dtype=np.float64) + 0.5 * h * (np.asarray(dom.dims) - 1)


def box_diagonal(dom, h):
    return float(np.linalg.norm(h * (np.asarray(dom.dims) - 1)))


def moments(dS, dom, h):
    """The 22 moments of dS [4][N] about the domain's centre (FP64)."""
    r = grid_points(dom, h) - box_centre(dom, h)[None, :]
    w = h ** 3
    rho, J = dS[0], dS[1:4]
    out = np.zeros(N_FEAT)
    out[0] = w * rho.sum()
    out[1:4] = w * (rho[:, None] * r).sum(axis=0)
    second = w * np.einsum("n,ni,nj->ij", rho, r, r)
    out[4:10] = [second[0, 0], second[1, 1], second[2, 2], second[0, 1], second[0, 2], second[1, 2]]
    out[10:13] = w * J.sum(axis=1)
    out[13:22] = (w * J @ r).ravel()            # K[i][j] = sum J_i x_j
    return out


# index triples of the 10 distinct third moments, in storage order
OCT = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 0, 1), (0, 0, 2), (0, 1, 1), (1, 1, 2), (0, 2, 2), (1, 2, 2), (0, 1, 2)]
# index pairs of the 6 distinct second moments (xx yy zz xy xz yz)
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def higher_moments(dS, dom, h):
    """The 28 further moments of dS [4][N] used by the analytic far field
    (weight h^3, about the box centre): the charge's third moments
    O_ijk = sum dS_0 x_i x_j x_k (10, in OCT order) and the current's second
    moments N_i,jk = sum dS_{1+i} x_j x_k (3 x 6, PAIRS order)."""
    r = grid_points(dom, h) - box_centre(dom, h)[None, :]
    w = h ** 3
    out = np.zeros(28)
    for k, (a, b, c) in enumerate(OCT):
        out[k] = w * np.sum(dS[0] * r[:, a] * r[:, b] * r[:, c])
    for i in range(3):
        for k, (a, b) in enumerate(PAIRS):
            out[10 + 6 * i + k] = w * np.sum(dS[1 + i] * r[:, a] * r[:, b])
    return out


def frame(d):
    """Rows e1, e2, e3 of the pair frame for d = c_target - c_source."""
    d = np.asarray(d, dtype=np.float64)
    e1 = d / np.linalg.norm(d)
    ref = np.array([1.0, 0.0, 0.0]) if abs(e1[2]) > 0.9 else np.array([0.0, 0.0, 1.0])
    e2 = ref - (ref @ e1) * e1
    e2 /= np.linalg.norm(e2)
    return np.stack([e1, e2, np.cross(e1, e2)])


def rotate(m, R):
    """Moments m [22] expressed in the frame with axes R (rows)."""
    out = np.zeros(N_FEAT)
    out[0] = m[0]
    out[1:4] = R @ m[1:4]
    Q = np.array([[m[4], m[7], m[8]], [m[7], m[5], m[9]], [m[8], m[9], m[6]]])
    Qr = R @ Q @ R.T
    out[4:10] = [Qr[0, 0], Qr[1, 1], Qr[2, 2], Qr[0, 1], Qr[0, 2], Qr[1, 2]]
    out[10:13] = R @ m[10:13]
    out[13:22] = (R @ m[13:22].reshape(3, 3) @ R.T).ravel()
    return out


def pair_geometry(system, s, n):
    """(d = c_s - c_n, |d|, m_c, frac) of the pair target s <- source n."""
    h = system.h
    d = box_centre(system.domains[s], h) - box_centre(system.domains[n], h)
    dist = float(np.linalg.norm(d))
    x = dist / (system.c * system.dt)
    m_c = int(math.floor(x + 0.5))
    return d, dist, m_c, x - m_c


def features(system, samples, s, n, l, n_lags):
    """Network input of pair (s <- n) at step l; samples[n][t] = S(t) [4][N]."""
    h = system.h
    d, dist, m_c, frac = pair_geometry(system, s, n)
    R = frame(d)
    dom = system.domains[n]
    H = np.zeros((n_lags, N_FEAT))
    for j in range(n_lags):
        m = m_c - n_lags // 2 + j
        t = l - m
        if t > 0 and m >= 0:
            H[j] = rotate(moments(samples[n][t] - samples[n][0], dom, h), R)
    dbar = np.mean([box_diagonal(dm, h) for dm in system.domains])
    g, f = 10.0 * dbar / dist, frac
    blocks = [H, g * H, f * H, g * f * H, g * g * H, f * f * H]
    return np.concatenate([b.ravel() for b in blocks] + [[g, f]])


def legendre(x):
    x = np.asarray(x, dtype=np.float64)
    return [np.ones_like(x), x, 0.5 * (3 * x * x - 1), 0.5 * x * (5 * x * x - 3)]


def basis(u):
    """[npts][20] basis values at points u [npts][3]."""
    px, py, pz = legendre(u[:, 0]), legendre(u[:, 1]), legendre(u[:, 2])
    return np.stack([px[i] * py[j] * pz[k] for i, j, k in DEGREES], axis=1)


def frame_coords(system, s, R):
    dom = system.domains[s]
    h = system.h
    ell = 0.5 * h * (max(dom.dims) - 1)
    r = grid_points(dom, h) - box_centre(dom, h)[None, :]
    return (r @ R.T) / ell


def box_coords(dom):
    axes = [np.linspace(-1.0, 1.0, n) for n in dom.dims]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def frame_fit(system, s, n, F):
    """Least-squares frame coefficients a [4][20] of a field F [4][N_s] on
    target s for the pair (s <- n); the A part is taken in frame components."""
    d, _, _, _ = pair_geometry(system, s, n)
    R = frame(d)
    B = basis(frame_coords(system, s, R))
    G = np.vstack([F[0][None, :], R @ F[1:4]])
    coef, *_ = np.linalg.lstsq(B, G.T, rcond=None)
    return coef.T


def frame_synth(system, s, n, a):
    """Field [4][N_s] of frame coefficients a [4][20] (inverse of frame_fit)."""
    d, _, _, _ = pair_geometry(system, s, n)
    R = frame(d)
    B = basis(frame_coords(system, s, R))
    G = (B @ a.T).T
    return np.vstack([G[0][None, :], R.T @ G[1:4]])


# ---------------------------------------------------------------------------
# Analytic multipole field of a far source (the non-learned far-pair path).
#
# With R the vector from the source centre to the target point, u = R/|R| and
# the source shape expanded about the centre, every term of the lag sum is
# F(t - |R - r'|/c) / |R - r'| with r' the source point.  Its Taylor expansion
# in r' is sum_n (-1)^n / n! (r'.grad)^n [F(t - R/c) / R], so the moment of
# order n multiplies the n-th gradient of the radial function
# g(R) = F(t - R/c)/R, whose R-derivatives are (F^(k): k-th time derivative)
#   g1 = -F/R^2 - F^(1)/(cR)
#   g2 = 2F/R^3 + 2F^(1)/(cR^2) + F^(2)/(c^2 R)
#   g3 = -6F/R^4 - 6F^(1)/(cR^3) - 3F^(2)/(c^2 R^2) - F^(3)/(c^3 R),
# and the gradients of a radial function are
#   d_i g = u_i g1,  d_ij g = u_i u_j (g2 - g1/R) + delta_ij g1/R,
#   d_ijk g = u_i u_j u_k (g3 - 3 g2/R + 3 g1/R^2) + (delta_ij u_k + ...)(g2/R - g1/R^2).
# Contracting with the charge moments to third order and the current moments
# to second order gives, with the time derivatives at t - R/c:
#   v   = q/R + u.p/R^2 + u.p^(1)/(cR)
#         + (3 u.Q.u - tr Q)/(2R^3) + (3 u.Q^(1).u - tr Q^(1))/(2cR^2) + u.Q^(2).u/(2c^2 R)
#         + (15 O_uuu - 9 u.trO)/(6R^4) + (15 O^(1)_uuu - 9 u.trO^(1))/(6cR^3)
#         + (6 O^(2)_uuu - 3 u.trO^(2))/(6c^2 R^2) + O^(3)_uuu/(6c^3 R)
#   A_i = J_i/R + u.K_i/R^2 + u.K_i^(1)/(cR)
#         + (3 u.N_i.u - tr N_i)/(2R^3) + (3 u.N_i^(1).u - tr N_i^(1))/(2cR^2)
#         + u.N_i^(2).u/(2c^2 R)
# (O_uuu = sum O_ijk u_i u_j u_k, (trO)_k = sum_i O_iik).  The moments between
# samples are cubic Lagrange interpolants of the four samples around the
# retarded time; the derivatives are those of the same cubic.

def _cubic_weights(u):
    """Value and first, second, third derivative weights (per step) at u in
    [0, 1) for samples at -1, 0, 1, 2."""
    x = np.array([-1.0, 0.0, 1.0, 2.0])
    w, d1, d2, d3 = np.zeros(4), np.zeros(4), np.zeros(4), np.zeros(4)
    for k in range(4):
        others = [x[j] for j in range(4) if j != k]
        den = np.prod([x[k] - o for o in others])
        # polynomial prod (u - o) / den: value and derivatives
        a, b, c_ = others
        w[k] = (u - a) * (u - b) * (u - c_) / den
        d1[k] = ((u - b) * (u - c_) + (u - a) * (u - c_) + (u - a) * (u - b)) / den
        d2[k] = 2.0 * ((u - a) + (u - b) + (u - c_)) / den
        d3[k] = 6.0 / den
    return w, d1, d2, d3


def _sym3(f):
    """Full 3x3x3 tensor from the 10 distinct third moments (OCT order)."""
    T = np.zeros((3, 3, 3))
    for k, (a, b, c) in enumerate(OCT):
        for idx in {(a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)}:
            T[idx] = f[k]
    return T


def _sym2(f):
    """Symmetric 3x3 matrix from (xx yy zz xy xz yz)."""
    return np.array([[f[0], f[3], f[4]], [f[3], f[1], f[5]], [f[4], f[5], f[2]]])


def multipole_field(system, samples, s, n, l, pts, order=3):
    """v and A [4][len(pts)] of source n at points pts [n][3] and step l
    (order=2: charge to second and current to first order only)."""
    h, dt, c = system.h, system.dt, system.c
    dom = system.domains[n]
    cn = box_centre(dom, h)
    mom = {}

    def m_at(t):
        if t <= 0:
            return np.zeros(N_FEAT + 28)
        if t not in mom:
            d = samples[n][t] - samples[n][0]
            mom[t] = np.concatenate([moments(d, dom, h), higher_moments(d, dom, h)])
        return mom[t]

    out = np.zeros((4, len(pts)))
    for k, r in enumerate(np.asarray(pts, dtype=np.float64)):
        Rv = r - cn
        R = float(np.linalg.norm(Rv))
        u = Rv / R
        tau = l - R / (c * dt)
        a = int(np.floor(tau))
        w, d1, d2, d3 = _cubic_weights(tau - a)
        F = np.stack([m_at(a - 1 + j) for j in range(4)])
        f = [w @ F, (d1 @ F) / dt, (d2 @ F) / dt ** 2, (d3 @ F) / dt ** 3]
        # the lag sum reads the sources through their linear interpolant (the
        # triangle basis), which lies on the chords: averaged over the spread of
        # retarded times across a source it is S + dt^2/12 S''.  The far terms
        # carry the same bias, so that they model the plain lag sum.
        f = [f[0] + dt * dt / 12.0 * f[2], f[1] + dt * dt / 12.0 * f[3], f[2], f[3]]

        def Qm(g):
            return np.array([[g[4], g[7], g[8]], [g[7], g[5], g[9]], [g[8], g[9], g[6]]])

        def oct_terms(g):
            T = _sym3(g[22:32])
            return np.einsum("ijk,i,j,k->", T, u, u, u), np.einsum("iik,k->", T, u)

        v = f[0][0] / R + u @ f[0][1:4] / R ** 2 + u @ f[1][1:4] / (c * R)
        v += (3 * u @ Qm(f[0]) @ u - np.trace(Qm(f[0]))) / (2 * R ** 3)
        v += (3 * u @ Qm(f[1]) @ u - np.trace(Qm(f[1]))) / (2 * c * R ** 2)
        v += (u @ Qm(f[2]) @ u) / (2 * c * c * R)
        K0, K1 = f[0][13:22].reshape(3, 3), f[1][13:22].reshape(3, 3)
        A = f[0][10:13] / R + K0 @ u / R ** 2 + K1 @ u / (c * R)
        out[0, k] = v
        out[1:4, k] = A
        if order < 3:
            continue
        o0, o1, o2, o3 = (oct_terms(g) for g in f)
        v += (15 * o0[0] - 9 * o0[1]) / (6 * R ** 4) + (15 * o1[0] - 9 * o1[1]) / (6 * c * R ** 3)
        v += (6 * o2[0] - 3 * o2[1]) / (6 * c * c * R ** 2) + o3[0] / (6 * c ** 3 * R)
        for i in range(3):
            N0, N1, N2 = (_sym2(g[32 + 6 * i: 38 + 6 * i]) for g in f[:3])
            A[i] += (3 * u @ N0 @ u - np.trace(N0)) / (2 * R ** 3)
            A[i] += (3 * u @ N1 @ u - np.trace(N1)) / (2 * c * R ** 2)
            A[i] += (u @ N2 @ u) / (2 * c * c * R)
        out[0, k] = v
        out[1:4, k] = A
    return out
