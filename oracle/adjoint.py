"""Objectives and the discrete adjoint of the RK4 forward map.

Oracle (test infrastructure only).

The paper obtains dJ/ds from the adjoint system (Eq. 6: forward LLG, adjoint
state a = dJ/dm integrated backwards from a(T) = dJ/dm(T)) and the gradient
integral (Eq. 7).  Here the same idea is applied to the *discrete* forward map:
the adjoint state after step n is lambda_n = dJ/dm_n, propagated backwards
through the transpose of each RK4 step, and the parameter gradient is the sum
over steps and stages of the stage adjoints contracted with the parameter
derivative of the right-hand side.  The result is the exact gradient of the
discrete objective.

RK4 step transpose, with lambda' = lambda_{n+1} and stage states y_s:
  l4 = dt/6 lambda'            mu4 = J_f(y4)^T l4
  l3 = dt/3 lambda' + dt mu4   mu3 = J_f(y3)^T l3
  l2 = dt/3 lambda' + dt/2 mu3 mu2 = J_f(y2)^T l2
  l1 = dt/6 lambda' + dt/2 mu2 mu1 = J_f(y1)^T l1
  lambda_n = lambda' + mu1 + mu2 + mu3 + mu4 (+ dJ/dm_n of a running cost)
  dJ/dpsi += sum_s l_s . df/dpsi(y_s)

Transpose of f(m) = -g' [m x B + alpha m x (m x B)] applied to v, with
w = v x m and c = m x B:
  u  = -g' (w + alpha w x m)                 (adjoint of the field)
  mu = -g' (B x v + alpha c x v + alpha B x w) + J_B^T u
and u . dB/dpsi gives the psi-gradient of the stage.
"""
from __future__ import annotations

import numpy as np

from .micromag import MU0, TERM_ANIS, TERM_DEMAG, TERM_EXCH, cross, dot

OBJ_NONE, OBJ_ENERGY_AREA, OBJ_PORT_MY2, OBJ_PORT_SPECTRAL, OBJ_MAG_CURVE = 0, 1, 2, 3, 4


class Objective:
    """kind: OBJ_ENERGY_AREA    -> J = (E_ex + E_d)(m_T)/E_ref + lam (mean psi - area)^2
             OBJ_PORT_MY2       -> J = 1/|W| sum_{n in W} [mean_P1 m_y^2 - mean_P2 m_y^2],
                                   W = {n : n_start < n <= n_steps}
             OBJ_PORT_SPECTRAL  -> J = sum_q coef[0, q] |X_1(f_q)| + coef[1, q] |X_2(f_q)|
                                   (Eq. 10 with its frequency windows; see spectral_value)
             OBJ_MAG_CURVE      -> J = sum_{n in W} weight_n |M_x(n) - target_n|,
                                   M_x the psi-weighted mean of m_x (Eq. 8;
                                   see curve_series)."""

    def __init__(self, kind, E_ref=1.0, lam=1.0, area=0.4, n_start=0, port1=None, port2=None, freqs=None,
                 coef=None, target=None, weight=None):
        self.kind = kind
        self.E_ref = E_ref
        self.lam = lam
        self.area = area
        self.n_start = n_start
        self.port1 = None if port1 is None else np.asarray(port1, float)
        self.port2 = None if port2 is None else np.asarray(port2, float)
        self.freqs = None if freqs is None else np.asarray(freqs, float)
        self.coef = None if coef is None else np.asarray(coef, float).reshape(2, -1)
        self.target = None if target is None else np.asarray(target, float)
        self.weight = None if weight is None else np.asarray(weight, float)


# -- objective values and their explicit derivatives --------------------------

def energy_area_value(sim, m, psi, obj):
    e = sim.energies(m, psi, 0.0, terms=sim.terms & (TERM_EXCH | TERM_DEMAG))
    return (e["ex"] + e["d"]) / obj.E_ref + obj.lam * (psi.mean() - obj.area) ** 2


def energy_area_grad(sim, m, psi, obj):
    """(dJ/dm, dJ/dpsi) of the energy + area objective, from the energy sums."""
    p = sim.p
    V = sim.V
    gm = np.zeros(m.shape, dtype=np.result_type(m, psi, float))
    gp = np.zeros(psi.shape, dtype=np.result_type(m, psi, float))
    if sim.terms & TERM_EXCH:
        for ax, h, a, b in sim._edges():
            pa, pb, s, nz = sim._pair(psi, ax, h)
            dm = m[b] - m[a]
            coef = np.where(nz, V * p.A * 2.0 * pa * pb / s, 0.0) / (h * h)
            gm[b] += 2.0 * coef * dm
            gm[a] -= 2.0 * coef * dm
            d2 = dot(dm, dm)
            sl_a = a[1:]
            sl_b = b[1:]
            gp[sl_a] += np.where(nz, V * p.A * 2.0 * pb * pb / (s * s), 0.0) * d2 / (h * h)
            gp[sl_b] += np.where(nz, V * p.A * 2.0 * pa * pa / (s * s), 0.0) * d2 / (h * h)
    if sim.terms & TERM_DEMAG:
        conv = sim.demag.conv(psi * m)
        gm = gm + MU0 * p.Ms ** 2 * V * psi * conv
        gp = gp + MU0 * p.Ms ** 2 * V * dot(m, conv)
    gm = gm / obj.E_ref
    gp = gp / obj.E_ref + 2.0 * obj.lam * (psi.mean() - obj.area) / psi.size
    return gm, gp


def port_value(m, obj):
    my2 = m[1] * m[1]
    return (my2 * obj.port1).sum() / obj.port1.sum() - (my2 * obj.port2).sum() / obj.port2.sum()


def port_source(m, obj, n_window):
    g = np.zeros(m.shape, dtype=m.dtype)
    g[1] = 2.0 * m[1] * (obj.port1 / obj.port1.sum() - obj.port2 / obj.port2.sum()) / n_window
    return g


# -- spectral port objective (Eq. 10) ------------------------------------------
#
# Eq. 10 compares, at the two outputs, sums of the magnitudes of the Fourier
# transform of the magnetisation oscillation over frequency windows around f1
# and f2.  Readings: the oscillation recorded at output j is the port-mean m_y
# of the states m_n of the window W = {n_start < n <= n_steps}, at t_n = t0 +
# n dt; its transform at frequency f is the plain (rectangular-window) DFT
# X_j(f) = 1/|W| sum_{n in W} x_j(n) exp(-2 pi i f t_n), evaluated at the
# sample frequencies f_q of the windows; J = sum_q c_1q |X_1(f_q)| + c_2q |X_2(f_q)|,
# where Eq. 10 takes c = +1 / -1 on the output that should / should not carry
# a window's frequency.  Real and imaginary parts are kept as separate sums, so
# that complex-step perturbations of the series pass through |X| analytically.

def port_series(traj, obj, n_steps):
    """x_j(n), n in W: the port-mean m_y of each output (shape (2, |W|))."""
    win = range(obj.n_start + 1, n_steps + 1)
    w1, w2 = obj.port1 / obj.port1.sum(), obj.port2 / obj.port2.sum()
    return np.array([[(traj[n][1] * w1).sum() for n in win], [(traj[n][1] * w2).sum() for n in win]])


def spectral_parts(x, times, freqs):
    """(C, S): C_jq = 1/|W| sum_n x_j(n) cos(2 pi f_q t_n), S likewise with sin;
    X_j(f_q) = C_jq - i S_jq."""
    th = 2 * np.pi * np.outer(freqs, times)          # (K, |W|)
    W = len(times)
    return x @ np.cos(th).T / W, x @ np.sin(th).T / W


def spectral_value(x, times, obj):
    C, S = spectral_parts(x, times, obj.freqs)
    return (obj.coef * np.sqrt(C * C + S * S)).sum()


def spectral_sources(x, times, obj):
    """dJ/dx_j(n) (shape (2, |W|)): d|X| = (C dC + S dS) / |X|, dC/dx(n) = cos/|W|, dS/dx(n) = sin/|W|."""
    C, S = spectral_parts(x, times, obj.freqs)
    A = np.sqrt(C * C + S * S)
    th = 2 * np.pi * np.outer(obj.freqs, times)
    W = len(times)
    wc = obj.coef * C / A
    ws = obj.coef * S / A
    return (wc @ np.cos(th) + ws @ np.sin(th)) / W


def spectral_source_field(g, m, obj):
    """dJ/dm_n of one window state from the series sources g = (g_1(n), g_2(n))."""
    out = np.zeros(m.shape, dtype=np.result_type(m, g))
    out[1] = g[0] * obj.port1 / obj.port1.sum() + g[1] * obj.port2 / obj.port2.sum()
    return out


# -- magnetisation-curve objective (Eq. 8) -------------------------------------
#
# Eq. 8 sums, over the steps of a run whose applied field ramps linearly from 0
# to 0.3 Ms, the distance between the particle's average magnetisation M_x and
# the target curve, each term divided by the target and by the number of steps.
# The Stoner-Wohlfarth section takes M_x as the particle's average x component:
# here M_x(n) = sum_i psi_i m_x,i(n) / sum_i psi_i (the material-weighted mean of
# m_x, in units of Ms; 0 when there is no material), for the states m_n of the
# window W.  The weights weight_n = 1 / (M^target_n N) and the target are inputs
# (the section's target is M = 2 H_ext, i.e. 0.6 n / N in units of Ms along the
# ramp; the n = 0 term, whose target is 0, is left out).  |.| takes the zero
# subgradient at 0.  J depends on psi explicitly through M_x:
#   dM_x(n)/dm_x,i = psi_i / S,   dM_x(n)/dpsi_i = (m_x,i(n) - M_x(n)) / S,
# with S = sum_i psi_i.

def _absr(z):
    """|z| for real z, continued analytically for complex-step perturbations."""
    return np.where(np.real(z) >= 0, z, -z)


def curve_series(traj, psi, obj, n_steps):
    """M_x(n) for the window states: the psi-weighted mean of m_x."""
    win = range(obj.n_start + 1, n_steps + 1)
    S = psi.sum()
    if np.real(S) == 0:
        return np.zeros(len(win), dtype=np.result_type(psi, traj[0]))
    return np.array([(psi * traj[n][0]).sum() / S for n in win])


def curve_value(M, obj):
    return (obj.weight * _absr(M - obj.target)).sum()


def curve_sources(M, obj):
    """dJ/dM(n) = weight_n sign(M(n) - target_n) (0 where they are equal)."""
    return obj.weight * np.sign(np.real(M - obj.target))


# -- transpose of one right-hand-side evaluation -------------------------------

def rhs_vjp(sim, m, B, psi, v):
    """(mu, g_psi): J_f(m)^T v and v . df/dpsi at the state m with field B."""
    gp_ = sim.gp
    al = sim.alpha
    frozen = sim.frozen(psi)
    w = cross(v, m)
    c = cross(m, B)
    u = -gp_ * (w + al * cross(w, m))
    u = np.where(frozen, 0.0, u)
    mu = -gp_ * (cross(B, v) + al * cross(c, v) + al * cross(B, w))
    mu = np.where(frozen, 0.0, mu)
    g = np.zeros(psi.shape, dtype=np.result_type(m, v, psi, float))
    if sim.terms & TERM_EXCH:
        k = sim.kappa
        for ax, h, a, b in sim._edges():
            pa, pb, s, nz = sim._pair(psi, ax, h)
            cab = np.where(nz, 2.0 * pb / (s * h * h), 0.0)
            cba = np.where(nz, 2.0 * pa / (s * h * h), 0.0)
            mu[a] += k * (cba * u[b] - cab * u[a])
            mu[b] += k * (cab * u[a] - cba * u[b])
            dm = m[b] - m[a]
            us = dot(u[a] + u[b], dm)
            sl_a = a[1:]
            sl_b = b[1:]
            g[sl_a] += np.where(nz, -k * 2.0 * pb / (s * s * h * h), 0.0) * us
            g[sl_b] += np.where(nz, k * 2.0 * pa / (s * s * h * h), 0.0) * us
    if sim.terms & TERM_DEMAG:
        cu = -MU0 * sim.p.Ms * sim.demag.conv(u)
        mu = mu + psi * cu
        g = g + dot(m, cu)
    if sim.terms & TERM_ANIS:
        coef = 2.0 * sim.p.K / sim.p.Ms
        uu = sim.u[:, None, None, None]
        mu = mu + coef * dot(u, uu) * uu
    return mu, g


# -- forward + objective + adjoint ---------------------------------------------

def window_times(sim, obj, n_steps, t0=0.0):
    return t0 + np.arange(obj.n_start + 1, n_steps + 1) * sim.p.dt


def objective_value(sim, traj, psi, obj, n_steps, t0=0.0):
    if obj.kind == OBJ_ENERGY_AREA:
        return energy_area_value(sim, traj[-1], psi, obj)
    if obj.kind == OBJ_PORT_MY2:
        win = range(obj.n_start + 1, n_steps + 1)
        return sum(port_value(traj[n], obj) for n in win) / len(win)
    if obj.kind == OBJ_PORT_SPECTRAL:
        return spectral_value(port_series(traj, obj, n_steps), window_times(sim, obj, n_steps, t0), obj)
    if obj.kind == OBJ_MAG_CURVE:
        return curve_value(curve_series(traj, psi, obj, n_steps), obj)
    return 0.0


def forward_objective(sim, m0, psi, n_steps, obj, t0=0.0):
    """J of the discrete forward map (stores the whole trajectory)."""
    m, traj = sim.integrate(m0, psi, n_steps, t0=t0, keep=True)
    return objective_value(sim, traj, psi, obj, n_steps, t0), traj


def gradient(sim, m0, psi, n_steps, obj, t0=0.0):
    """J, dJ/dpsi and dJ/dm0 by the discrete adjoint (store-all trajectory)."""
    dt = sim.p.dt
    J, traj = forward_objective(sim, m0, psi, n_steps, obj, t0)
    n_window = max(1, n_steps - obj.n_start)
    lam = np.zeros(m0.shape, dtype=np.result_type(m0, psi, float))
    g_psi = np.zeros(psi.shape, dtype=np.result_type(m0, psi, float))
    if obj.kind == OBJ_ENERGY_AREA:
        gm, gp = energy_area_grad(sim, traj[-1], psi, obj)
        lam = lam + gm
        g_psi = g_psi + gp
    if obj.kind == OBJ_PORT_MY2 and n_steps > obj.n_start:
        lam = lam + port_source(traj[n_steps], obj, n_window)
    spec = obj.kind == OBJ_PORT_SPECTRAL and n_steps > obj.n_start
    if spec:
        g_ser = spectral_sources(port_series(traj, obj, n_steps), window_times(sim, obj, n_steps, t0), obj)
        lam = lam + spectral_source_field(g_ser[:, -1], traj[n_steps], obj)
    curve = obj.kind == OBJ_MAG_CURVE and n_steps > obj.n_start
    if curve:
        # with c_n = dJ/dM(n) / S: dJ/dm_x,i(n) = c_n psi_i and dJ/dpsi_i += c_n (m_x,i(n) - M(n))
        M_cur = curve_series(traj, psi, obj, n_steps)
        S = psi.sum()
        g_cur = curve_sources(M_cur, obj) / S if np.real(S) != 0 else np.zeros_like(M_cur)

        def curve_terms(g, m, M):
            gm = np.zeros(m.shape, dtype=np.result_type(m, psi, g))
            gm[0] = g * psi
            return gm, g * (m[0] - M)
        gm, gp = curve_terms(g_cur[-1], traj[n_steps], M_cur[-1])
        lam = lam + gm
        g_psi = g_psi + gp
    for n in range(n_steps - 1, -1, -1):
        t = t0 + n * dt
        _, ys, Bs = sim.rk4_step(traj[n], psi, t)
        l4 = dt / 6.0 * lam
        mu4, g4 = rhs_vjp(sim, ys[3], Bs[3], psi, l4)
        l3 = dt / 3.0 * lam + dt * mu4
        mu3, g3 = rhs_vjp(sim, ys[2], Bs[2], psi, l3)
        l2 = dt / 3.0 * lam + 0.5 * dt * mu3
        mu2, g2 = rhs_vjp(sim, ys[1], Bs[1], psi, l2)
        l1 = dt / 6.0 * lam + 0.5 * dt * mu2
        mu1, g1 = rhs_vjp(sim, ys[0], Bs[0], psi, l1)
        lam = lam + mu1 + mu2 + mu3 + mu4
        g_psi = g_psi + g1 + g2 + g3 + g4
        if obj.kind == OBJ_PORT_MY2 and obj.n_start < n <= n_steps:
            lam = lam + port_source(traj[n], obj, n_window)
        if spec and obj.n_start < n:
            lam = lam + spectral_source_field(g_ser[:, n - obj.n_start - 1], traj[n], obj)
        if curve and obj.n_start < n:
            k = n - obj.n_start - 1
            gm, gp = curve_terms(g_cur[k], traj[n], M_cur[k])
            lam = lam + gm
            g_psi = g_psi + gp
    return J, g_psi, lam
