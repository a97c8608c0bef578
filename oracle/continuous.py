"""Continuous adjoint (Eqs. 6-7): the adjoint equation integrated backwards in
time, as the paper's torchdiffeq-based solver does, for comparison with the
discrete adjoint.

Oracle (test infrastructure only).

Eq. 6 carries a(t) = dJ/dm(t) backwards from a(T) = dJ/dm(T) with
da/dt = -J_f(m(t))^T a, and Eq. 7 collects dJ/dpsi = integral of a . df/dpsi.
Readings: the augmented system (a, dJ/dpsi) is integrated with classic RK4
backwards over each interval [t_n, t_n+1] of a forward run whose states m_n are
kept; the forward state at the interval's midpoint is the cubic Hermite
interpolant m_mid = (m_n + m_n+1)/2 + h/8 (f(m_n) - f(m_n+1)) (fourth-order
accurate), so that the Jacobians are taken on the trajectory and not on the
forward integrator's stage states.  Per interval, with G(A, m) = J_f(m)^T A:
  A1 = a_n+1, A2 = a_n+1 + h/2 G1, A3 = a_n+1 + h/2 G2, A4 = a_n+1 + h G3,
  a_n = a_n+1 + h/6 (G1 + 2 G2 + 2 G3 + G4), the states m_n+1, m_mid, m_mid, m_n,
and dJ/dpsi gains h/6 (q1 + 2 q2 + 2 q3 + q4), q_s = A_s . df/dpsi(m_s).
The paper's adjoint solve chooses its own steps.  Here the backward pass may
split each interval into n_sub equal RK4 sub-steps, with the states inside the
interval taken from the same cubic Hermite interpolant
  m(t_n + th h) = h00 m_n + h10 h f(m_n) + h01 m_n+1 + h11 h f(m_n+1),
  h00 = 2th^3 - 3th^2 + 1, h10 = th^3 - 2th^2 + th, h01 = 3th^2 - 2th^3,
  h11 = th^3 - th^2
(th = 1/2 gives the midpoint above).  Sub-steps matter on stiff problems: an
adaptive Dormand-Prince run settles where its own stability region ends, which
lies beyond classic RK4's, so RK4 on the forward steps can diverge there.
The result approaches the discrete adjoint's as the steps shrink.
"""
from __future__ import annotations

from .adjoint import rhs_vjp


def hermite(m0, m1, f0, f1, h, th):
    """Cubic Hermite interpolant on [t_n, t_n + h] at t_n + th h."""
    h00 = 2.0 * th ** 3 - 3.0 * th ** 2 + 1.0
    h10 = th ** 3 - 2.0 * th ** 2 + th
    h01 = 3.0 * th ** 2 - 2.0 * th ** 3
    h11 = th ** 3 - th ** 2
    return h00 * m0 + (h10 * h) * f0 + h01 * m1 + (h11 * h) * f1


def rk4_back(sim, psi, a, gpsi, h, up, mid, lo):
    """One classic RK4 step of (a, dJ/dpsi) backwards over h, with the
    Jacobians at the (state, field) pairs up (the step's end), mid and lo."""
    G1, q1 = rhs_vjp(sim, up[0], up[1], psi, a)
    A2 = a + 0.5 * h * G1
    G2, q2 = rhs_vjp(sim, mid[0], mid[1], psi, A2)
    A3 = a + 0.5 * h * G2
    G3, q3 = rhs_vjp(sim, mid[0], mid[1], psi, A3)
    A4 = a + h * G3
    G4, q4 = rhs_vjp(sim, lo[0], lo[1], psi, A4)
    return (a + h / 6.0 * (G1 + 2.0 * G2 + 2.0 * G3 + G4),
            gpsi + h / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4))


def continuous_adjoint(sim, traj, ts, hs, psi, lam_T, gpsi_T, n_sub=1):
    """(dJ/dpsi, dJ/dm0) from the kept states traj[n] at ts[n] (steps hs),
    with n_sub RK4 sub-steps per interval."""
    if n_sub < 1:
        raise ValueError("n_sub must be >= 1")
    a, gpsi = lam_T, gpsi_T
    f_next, B_next = sim.rhs(traj[-1], psi, ts[-1])
    for n in range(len(hs) - 1, -1, -1):
        h = hs[n]
        m0_, m1_ = traj[n], traj[n + 1]
        f0, B0 = sim.rhs(m0_, psi, ts[n])

        def state(th):
            m = hermite(m0_, m1_, f0, f_next, h, th)
            return m, sim.rhs(m, psi, ts[n] + th * h)[1]
        up = (m1_, B_next)
        for k in range(n_sub - 1, -1, -1):
            mid = state((k + 0.5) / n_sub)
            lo = (m0_, B0) if k == 0 else state(k / n_sub)
            a, gpsi = rk4_back(sim, psi, a, gpsi, h / n_sub, up, mid, lo)
            up = lo
        f_next, B_next = f0, B0
    return gpsi, a
