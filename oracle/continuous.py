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
The result approaches the discrete adjoint's as the steps shrink.
"""
from __future__ import annotations

from .adjoint import rhs_vjp


def continuous_adjoint(sim, traj, ts, hs, psi, lam_T, gpsi_T):
    """(dJ/dpsi, dJ/dm0) from the kept states traj[n] at ts[n] (steps hs)."""
    a, gpsi = lam_T, gpsi_T
    f_next, B_next = sim.rhs(traj[-1], psi, ts[-1])
    for n in range(len(hs) - 1, -1, -1):
        h = hs[n]
        m0_, m1_ = traj[n], traj[n + 1]
        f0, B0 = sim.rhs(m0_, psi, ts[n])
        m_mid = 0.5 * (m0_ + m1_) + h / 8.0 * (f0 - f_next)
        _, B_mid = sim.rhs(m_mid, psi, ts[n] + 0.5 * h)
        G1, q1 = rhs_vjp(sim, m1_, B_next, psi, a)
        A2 = a + 0.5 * h * G1
        G2, q2 = rhs_vjp(sim, m_mid, B_mid, psi, A2)
        A3 = a + 0.5 * h * G2
        G3, q3 = rhs_vjp(sim, m_mid, B_mid, psi, A3)
        A4 = a + h * G3
        G4, q4 = rhs_vjp(sim, m0_, B0, psi, A4)
        a = a + h / 6.0 * (G1 + 2.0 * G2 + 2.0 * G3 + G4)
        gpsi = gpsi + h / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4)
        f_next, B_next = f0, B0
    return gpsi, a
