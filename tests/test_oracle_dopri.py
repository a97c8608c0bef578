"""Pins of the oracle's adaptive Dormand-Prince integrator and its adjoint:
fifth-order convergence and a fourth-order error estimate on the damped
macrospin's exact solution, tolerance-controlled global error, the
controller's accept / reject behaviour, and the discrete adjoint of the
accepted steps against complex-step directional derivatives."""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import dopri
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl

GAMMA = 1.76e11
H_CS = 1e-30


def macrospin(alpha=0.1, B=1.0):
    p = wl.Problem(nx=1, ny=1, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=8e5, A=1.3e-11, gamma=GAMMA, alpha0=alpha,
                   alpha_max=alpha, B0=(B, 0, 0), terms=wl.TERM_ZEEMAN, dt=1e-13)
    th0, ph0 = 1.0, 0.3
    m0 = np.array([math.cos(th0), math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0)]).reshape(3, 1, 1, 1)

    def exact(t):
        gp = GAMMA / (1 + alpha ** 2)
        th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * gp * B * t))
        ph = ph0 + gp * B * t
        return np.array([math.cos(th), math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph)])
    return mm.Sim(p), m0, np.ones((1, 1, 1)), exact


def test_fixed_steps_converge_at_fifth_order():
    sim, m0, psi, exact = macrospin()
    T = 2e-10
    errs = []
    for n in (400, 800):
        m = dopri.integrate_fixed(sim, m0, psi, 0.0, [T / n] * n)
        errs.append(np.abs(m[:, 0, 0, 0] - exact(T)).max())
    assert errs[1] < 1e-9
    assert 24.0 < errs[0] / errs[1] < 40.0     # 2^5 = 32


def test_embedded_estimate_is_fourth_order_per_step():
    """The local error estimate |y5 - y4| of one step shrinks as h^5."""
    sim, m0, psi, exact = macrospin()
    est = []
    for h in (2e-12, 1e-12):
        _, err, _ = dopri.dp_step(sim, m0, psi, 0.0, h, rtol=0.0, atol=1.0)
        est.append(err)
    assert 26.0 < est[0] / est[1] < 38.0


@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_adaptive_run_meets_its_tolerance(tol):
    sim, m0, psi, exact = macrospin()
    T = 2e-10
    m, hs, rej = dopri.integrate_adaptive(sim, m0, psi, 0.0, T, 1e-13, rtol=tol, atol=tol)
    assert abs(sum(hs) - T) <= 1e-24
    err = np.abs(m[:, 0, 0, 0] - exact(T)).max()
    assert err < 50 * tol
    # every accepted step passes the controller's test when replayed
    mm_, t = m0, 0.0
    for h in hs:
        y5, e, _ = dopri.dp_step(sim, mm_, psi, t, h, tol, tol)
        assert e <= 1.0
        mm_, t = y5, t + h


def test_controller_rejects_a_step_that_is_too_large():
    sim, m0, psi, exact = macrospin()
    m, hs, rej = dopri.integrate_adaptive(sim, m0, psi, 0.0, 2e-11, 1e-11, rtol=1e-10, atol=1e-10)
    assert rej >= 1 and hs[0] < 1e-11


def test_adjoint_of_the_accepted_steps_matches_complex_step():
    p = wl.Problem(nx=6, ny=5, nz=1, dx=3e-9, dy=3e-9, dz=4e-9, Ms=8e5, A=1.3e-11, K=5e4, ku=(0.6, 0.8, 0.0),
                   alpha0=0.2, alpha_max=0.2, B0=(0.05, 0.02, 0.1), b_rf=(0.0, 0.01, 0.0), f1=5e9,
                   terms=wl.TERM_ALL, dt=5e-14)
    rng = np.random.default_rng(12)
    sh = p.shape
    ant = np.zeros(sh)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((p.ny, p.nx)) * 0.5
    design = np.ones(sh)
    psif = np.zeros(sh)
    m0 = rng.standard_normal((3,) + sh)
    m0 /= np.sqrt((m0 ** 2).sum(0))
    sim = mm.Sim(p, antenna=ant)
    a = 3.0
    psi = ls.levelset_to_psi(phi, a, design, psif)
    _, hs, _ = dopri.integrate_adaptive(sim, m0, psi, 0.0, 2e-12, 5e-14, rtol=1e-6, atol=1e-6)
    assert len(hs) >= 5 and len(set(hs)) > 1
    obj = adj.Objective(adj.OBJ_ENERGY_AREA, E_ref=1e-18, lam=0.7, area=0.4)
    J, gpsi, lam0 = dopri.gradient_fixed(sim, m0, psi, 0.0, hs, obj)
    gphi = ls.levelset_vjp(phi, a, design, gpsi)

    def Jof(m0_, psi_):
        return adj.energy_area_value(sim, dopri.integrate_fixed(sim, m0_, psi_, 0.0, hs), psi_, obj)
    for _ in range(2):
        v = rng.standard_normal(phi.shape)
        d_cs = Jof(m0.astype(complex), ls.levelset_to_psi(phi + 1j * H_CS * v, a, design, psif)).imag / H_CS
        assert abs(d_cs - (gphi * v).sum()) <= 1e-11 * abs(d_cs)
        w = rng.standard_normal(m0.shape)
        d_cs = Jof(m0 + 1j * H_CS * w, psi.astype(complex)).imag / H_CS
        assert abs(d_cs - (lam0 * w).sum()) <= 1e-11 * abs(d_cs)
