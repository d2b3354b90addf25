"""FP64 reference of the toy propagation loop around the potential evaluation.

Test infrastructure: only tests/, the smoke check and the bench's CPU baseline
use this module.  It shares no code with the HIP path.

The paper's loop (Fig. 4) alternates the Kohn-Sham propagation, which gives
new sources, with the evaluation of the retarded potentials, which enter the
next propagation step; the current of step l drives the vector potential of
step l + 1 (Sec. II, the remark after the current density).  Without Kohn-Sham
orbitals the sources here are Lorentz oscillators: source k of a domain has
the fixed shape B_k = (B_rho, B_J) (a +/- Gaussian charge pair and its line
current, B_J already divided by c) and the amplitude q_k(t), so that

    S(r, t) = sum_k ( q_k B_rho_k(r), qdot_k B_J_k(r) ).

The force on q_k is the generalised force of the potentials on that shape,
from the interaction Lagrangian  -int rho v + int (J/c) . A:

    phi_k = h^3 sum_r B_rho_k . v,   psi_k = h^3 sum_r B_J_k . A,
    F_k   = -phi_k - d psi_k / dt + drive_k e_ext(t)

(for a uniform field E this is l_k . E, l_k the pair's dipole per unit q), and

    qddot + gamma qdot + omega^2 q = kappa F.

Time stepping (explicit, one step behind the potentials as in the paper's
loop): with the potentials of step l,
    F(l)       = -phi(l) - (psi(l) - psi(l-1)) / dt + drive e_ext(l dt)
                 (psi(-1) = psi(0): the history before step 0 is constant),
    qdot(l+1)  = qdot(l) + dt (kappa F(l) - gamma qdot(l) - omega^2 q(l)),
    q(l+1)     = q(l) + dt qdot(l+1)          (semi-implicit Euler),
and S(l + 1) from q(l + 1), qdot(l + 1).
"""
from __future__ import annotations

import numpy as np

from .ref import potential_full


def project(basis, P, h):
    """phi [K], psi [K] of the shapes basis [K][4][N] in the potential P [4][N]."""
    w = h ** 3
    phi = w * (basis[:, 0, :] @ P[0])
    psi = w * np.einsum("kan,an->k", basis[:, 1:4, :], P[1:4])
    return phi, psi


def synthesize(basis, q, qd):
    """S [4][N] of amplitudes q, qdot [K]."""
    S = np.empty((4, basis.shape[2]))
    S[0] = q @ basis[:, 0, :]
    S[1:4] = np.einsum("k,kan->an", qd, basis[:, 1:4, :])
    return S


def advance(q, qd, phi, psi, psi_prev, e_ext, params, dt):
    """One semi-implicit Euler step; params [K][4] = omega, gamma, kappa, drive."""
    omega, gamma, kappa, drive = (params[:, i] for i in range(4))
    F = -phi - (psi - psi_prev) / dt + drive * e_ext
    qd1 = qd + dt * (kappa * F - gamma * qd - omega * omega * q)
    return q + dt * qd1, qd1


def run_loop(system, bases, params, e_ext, L, q0=None, qd0=None):
    """The coupled loop for steps 0..L on the direct-sum potentials.

    bases[n] [K_n][4][N_n], params[n] [K_n][4], e_ext(t) the external field
    amplitude.  Returns per domain the arrays q, qdot, phi, psi [L+1][K_n]
    (state and projections at each step) and the sources S [L+1][4][N_n]."""
    nd = len(system.domains)
    dt, h = system.dt, system.h
    q = [np.zeros(len(b)) if q0 is None else np.array(q0[n], float) for n, b in enumerate(bases)]
    qd = [np.zeros(len(b)) if qd0 is None else np.array(qd0[n], float) for n, b in enumerate(bases)]
    S = [np.zeros((L + 1, 4, b.shape[2])) for b in bases]
    rec = {k: [np.zeros((L + 1, len(b))) for b in bases] for k in ("q", "qdot", "phi", "psi")}
    psi_prev = [None] * nd
    for n in range(nd):
        S[n][0] = synthesize(bases[n], q[n], qd[n])
    for l in range(L + 1):
        P = potential_full(system, [S[n][: l + 1] for n in range(nd)], [l])[0]
        for n in range(nd):
            phi, psi = project(bases[n], P[n], h)
            if psi_prev[n] is None:
                psi_prev[n] = psi
            rec["q"][n][l], rec["qdot"][n][l] = q[n], qd[n]
            rec["phi"][n][l], rec["psi"][n][l] = phi, psi
            q[n], qd[n] = advance(q[n], qd[n], phi, psi, psi_prev[n], e_ext(l * dt), params[n], dt)
            psi_prev[n] = psi
            if l < L:
                S[n][l + 1] = synthesize(bases[n], q[n], qd[n])
    rec["S"] = S
    return rec

