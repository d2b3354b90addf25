"""Pins of the coupled-loop oracle (CPU): the projection against closed forms
in uniform fields, the oscillator update against an accurate ODE solution, and
the whole loop against the far field of a point dipole acting on a
polarisable molecule (the paper's own check of the coupling, Sec. IV:
induced dipole = polarisability x the dipole field of the driven molecule)."""
import math

import numpy as np
from scipy.integrate import solve_ivp

import oracle
from oracle import coupled_ref as cr
from synth import sources as sy


def _one_pair_domain(n, h, centre, cp, cm, s):
    dom = sy.Domain((n, n, n), np.asarray(centre, float) - 0.5 * h * (n - 1))
    dom.charges.append(sy.Charge("pair", s, np.asarray(cp, float) + centre, np.asarray(cm, float) + centre,
                                 ("const", 0.0)))
    return dom


def test_projection_in_uniform_fields():
    """v = -E.r and a uniform A: phi = -E.l and psi = A.l / c, l = c+ - c-."""
    h, c = 0.2, sy.C_AU
    cp, cm = np.array([0.1, 0.2, 0.6]), np.array([-0.1, -0.1, -0.5])
    dom = _one_pair_domain(32, h, np.zeros(3), cp, cm, 0.5)
    B = sy.pair_shapes(dom, h, c)
    r = sy.grid_points(dom, h)
    E = np.array([0.3, -0.7, 1.1])
    A = np.array([0.2, 0.5, -0.4])
    P = np.zeros((4, len(r)))
    P[0] = -(r @ E) + 3.0                      # a constant offset does not act on a neutral pair
    P[1:4] = A[:, None]
    phi, psi = cr.project(B, P, h)
    ell = cp - cm
    assert abs(phi[0] + E @ ell) < 1e-6 * abs(E @ ell)
    assert abs(psi[0] - A @ ell / c) < 1e-6 * abs(A @ ell / c)
    # the force of a static uniform field is l . E
    q1, qd1 = cr.advance(np.zeros(1), np.zeros(1), phi, psi, psi, 0.0, np.array([[0.0, 0.0, 1.0, 0.0]]), 1.0)
    assert abs(qd1[0] - E @ ell) < 1e-6 * abs(E @ ell) and q1[0] == qd1[0]


def test_oscillator_update_converges_to_the_ode():
    """Driven damped oscillators with no potentials: semi-implicit Euler is
    first order; its error halves with dt."""
    params = np.array([[2.0, 0.1, 1.5, 0.8], [5.0, 0.0, 1.0, -1.2], [0.7, 0.5, 2.0, 0.3]])
    w_d = 1.3

    def e_ext(t):
        return math.sin(w_d * t)

    T = 6.0

    def rhs(t, y):
        q, qd = y[:3], y[3:]
        om, ga, ka, dr = params.T
        return np.concatenate([qd, ka * dr * e_ext(t) - ga * qd - om * om * q])

    exact = solve_ivp(rhs, (0, T), np.zeros(6), rtol=1e-12, atol=1e-14).y[:3, -1]
    errs = []
    for n_steps in (6000, 12000):
        dt = T / n_steps
        q, qd = np.zeros(3), np.zeros(3)
        z = np.zeros(3)
        for l in range(n_steps):
            q, qd = cr.advance(q, qd, z, z, z, e_ext(l * dt), params, dt)
        errs.append(np.max(np.abs(q - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 5e-3, errs
    assert 1.6 < errs[0] / errs[1] < 2.4, errs


def _far_field_case(dt, L, d=60.0, h=0.4):
    """Run the loop for two one-pair molecules d apart along y; return the
    loop's q1 and the reference oscillator's q1 with and without the vector
    potential term."""
    c = sy.C_AU
    cp, cm = np.array([0.0, 0.0, 0.5]), np.array([0.0, 0.0, -0.5])
    doms = [_one_pair_domain(8, h, np.array([0.0, 0.0, 0.0]), cp, cm, 0.6),
            _one_pair_domain(8, h, np.array([0.0, d, 0.0]), cp, cm, 0.6)]
    system = sy.System(h, dt, c, doms)
    bases = [sy.pair_shapes(dm, h, c) for dm in doms]
    params = [np.array([[6.0, 0.2, 1.0, 1.0]]), np.array([[9.0, 0.1, 1.0, 0.0]])]
    w_d, T_env = 3.0, 4.0

    def e_ext(t):
        return math.sin(math.pi * t / T_env) ** 2 * math.sin(w_d * t) if t < T_env else 0.0

    rec = cr.run_loop(system, bases, params, e_ext, L)
    # discrete dipoles per unit q: of the charge shape, and of the current
    # shape per unit dq/dt (equal in the continuum, not on a truncated box)
    lr = [h ** 3 * b[0, 0] @ sy.grid_points(dm, h) for b, dm in zip(bases, doms)]
    lj = [h ** 3 * c * b[0, 1:4].sum(axis=1) for b in bases]
    assert abs(lr[0][2] - 1.0) < 0.05 and abs(lj[0][2] - 1.0) < 0.05 and abs(lr[0][0]) < 1e-12
    # static self-field of molecule 1: phi_self = C_self q
    P_self = oracle.potential_full(sy.System(h, dt, c, [doms[1]]), [bases[1][0][None]], [0])[0][0]
    C_self = h ** 3 * bases[1][0, 0] @ P_self[0]
    assert C_self > 0
    # the point-dipole field of molecule 0 at molecule 1 from the loop's
    # history, read like the method reads it (linear in time between samples)
    q0, qd0 = rec["q"][0][:, 0], rec["qdot"][0][:, 0]
    t = np.arange(L + 1) * dt
    tr = t - d / c
    j = np.floor(tr / dt).astype(int)
    D = lr[0][2] * np.interp(tr, t, q0, left=0.0)
    Dd = lr[0][2] * np.where(j >= 0, (q0[np.clip(j + 1, 0, L)] - q0[np.clip(j, 0, L)]) / dt, 0.0)
    grad_part = -D / d ** 3 - Dd / (c * d * d)                      # -d_z v
    A_z = lj[0][2] * np.interp(tr, t, qd0, left=0.0) / (c * d)
    psi = lj[1][2] * A_z / c
    om, ga, ka, _ = params[1][0]

    def oscillator(with_a):
        q, qd = 0.0, 0.0
        out = np.zeros(L + 1)
        for l in range(L + 1):
            out[l] = q
            F = lr[1][2] * grad_part[l] - C_self * q
            if with_a:
                F -= (psi[l] - psi[max(l - 1, 0)]) / dt
            qd = qd + dt * (ka * F - ga * qd - om * om * q)
            q = q + dt * qd
        return out

    return rec["q"][1][:, 0], oscillator(True), oscillator(False)


def test_loop_reproduces_the_far_field_polarisability_response():
    """Molecule 0 is driven by an external pulse along z; molecule 1, 60 bohr
    away along y, only feels molecule 0's field.  Its response from the full
    loop must approach that of an oscillator driven by the retarded field of
    the point dipole D0(t) = q0(t) l0 (static, induction and radiation terms):
        -d_z v = -D0(t_r)/d^3 - D0'(t_r)/(c d^2),  A_z = D0'(t_r)/(c d),
    t_r = t - d/c, its own static self-field included.  The two time
    discretisations agree to first order in dt."""
    errs = []
    for dt, L in ((0.02, 300), (0.01, 600)):
        got, ref, no_a = _far_field_case(dt, L)
        scale = np.max(np.abs(ref))
        assert scale > 0
        errs.append((np.max(np.abs(got - ref)) / scale, np.max(np.abs(got - no_a)) / scale))
    (e1, na1), (e2, na2) = errs
    assert e1 < 2.5e-2, errs
    assert e2 < 0.6 * e1, errs
    # the radiation term matters: without A the answer is off by far more
    assert min(na1, na2) > 30 * e2, errs
