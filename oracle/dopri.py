"""Adaptive Dormand-Prince 5(4) integration of the LLG right-hand side and the
discrete adjoint of its accepted steps.

Oracle (test infrastructure only).

The Methods integrate the LLG equation with an adaptive step size.  Readings:
the embedded explicit Runge-Kutta pair of Dormand and Prince (1980), fifth
order carried forward, fourth order for the error estimate; the error norm is
the largest, over all nodes and components, of |y5 - y4| / (atol + rtol
max(|y_n|, |y_n+1|)) (a max-norm, so that it does not depend on the order of
a sum); a step is accepted when the norm is at most 1; the next step is h
times min(5, max(0.2, 0.9 norm^(-1/5))) (no growth right after a rejection),
clipped so that the run ends exactly at t_end.  The adjoint differentiates the
map of the accepted steps with their sizes held fixed (the controller's
choices are not differentiated).
"""
from __future__ import annotations

import numpy as np

from .adjoint import OBJ_ENERGY_AREA, energy_area_grad, energy_area_value, rhs_vjp

# Dormand & Prince (1980): nodes c, coefficients a (rows 2..7), weights of the
# fifth-order (b5) and fourth-order (b4) solutions.
C = (0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0)
A = ((),
     (1 / 5,),
     (3 / 40, 9 / 40),
     (44 / 45, -56 / 15, 32 / 9),
     (19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729),
     (9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656),
     (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84))
B5 = (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0)
B4 = (5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40)


def dp_stages(sim, m, psi, t, h):
    """Stage states Y_s, rates k_s and fields B_s (s = 1..7) of one step."""
    Ys, ks, Bs = [], [], []
    for s in range(7):
        Y = m
        for j, a in enumerate(A[s]):
            if a != 0.0:
                Y = Y + h * a * ks[j]
        k, B = sim.rhs(Y, psi, t + C[s] * h)
        Ys.append(Y)
        ks.append(k)
        Bs.append(B)
    return Ys, ks, Bs


def dp_step(sim, m, psi, t, h, rtol, atol):
    """(y5, error norm, stages) of one trial step."""
    Ys, ks, Bs = dp_stages(sim, m, psi, t, h)
    y5 = m + h * sum(b * k for b, k in zip(B5, ks) if b != 0.0)
    e = h * sum((b5 - b4) * k for b5, b4, k in zip(B5, B4, ks))
    scale = atol + rtol * np.maximum(np.abs(np.real(m)), np.abs(np.real(y5)))
    return y5, float(np.max(np.abs(np.real(e)) / scale)), (Ys, ks, Bs)


def step_factor(err, accepted_last):
    f = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.9 * err ** -0.2))
    return min(f, 1.0) if not accepted_last else f


def integrate_adaptive(sim, m0, psi, t0, t_end, h0, rtol, atol, max_steps=100000):
    """(m(t_end), accepted step sizes, number of rejected trials)."""
    m, t, h = m0, t0, h0
    hs, rejected, ok_last = [], 0, True
    while t < t_end:
        if len(hs) >= max_steps:
            raise RuntimeError("too many steps")
        h = min(h, t_end - t)
        y5, err, _ = dp_step(sim, m, psi, t, h, rtol, atol)
        if err <= 1.0:
            m = y5
            t = t + h if t_end - t > h else t_end
            hs.append(h)
            h = h * step_factor(err, ok_last)
            ok_last = True
        else:
            rejected += 1
            h = h * step_factor(err, False)
            ok_last = False
    return m, hs, rejected


def integrate_fixed(sim, m0, psi, t0, hs, keep=False):
    """The map of a given sequence of steps (t advances by each h)."""
    m, t = m0, t0
    traj = [m0]
    for h in hs:
        Ys, ks, _ = dp_stages(sim, m, psi, t, h)
        m = m + h * sum(b * k for b, k in zip(B5, ks) if b != 0.0)
        t = t + h
        if keep:
            traj.append(m)
    return (m, traj) if keep else m


def gradient_fixed(sim, m0, psi, t0, hs, obj):
    """J, dJ/dpsi and dJ/dm0 of the terminal energy objective through the
    fixed-step map: per step (y' = y + h sum_s b_s k_s, k_s = f(Y_s)),
    kappa_s = h (b_s lambda' + sum_{i>s} a_is mu_i), mu_s = J_f(Y_s)^T kappa_s,
    lambda = lambda' + sum_s mu_s, dJ/dpsi += sum_s kappa_s . df/dpsi(Y_s)."""
    if obj.kind != OBJ_ENERGY_AREA:
        raise ValueError("the adaptive path carries the terminal energy objective")
    mT, traj = integrate_fixed(sim, m0, psi, t0, hs, keep=True)
    J = energy_area_value(sim, mT, psi, obj)
    lam, g_psi = energy_area_grad(sim, mT, psi, obj)
    ts = [t0]
    for h in hs:
        ts.append(ts[-1] + h)                # the same additions as the forward run
    for n in range(len(hs) - 1, -1, -1):
        h = hs[n]
        Ys, _, Bs = dp_stages(sim, traj[n], psi, ts[n], h)
        mus = [None] * 7
        lam_new = lam
        for s in range(5, -1, -1):           # stage 7 has b = 0 and feeds no later stage
            kap = h * B5[s] * lam
            for i in range(s + 1, 6):
                a = A[i][s]
                if a != 0.0:
                    kap = kap + h * a * mus[i]
            mu, g = rhs_vjp(sim, Ys[s], Bs[s], psi, kap)
            mus[s] = mu
            lam_new = lam_new + mu
            g_psi = g_psi + g
        lam = lam_new
    return J, g_psi, lam
