"""Pins of the oracle's magnetisation-curve objective (Eq. 8) and the field
ramp: the Stoner-Wohlfarth hard-axis law under a slow ramp, M_x as the
particle's average (invariant to a uniform psi, the plain mean over the nodes
of a binary particle), the paper's target, and the discrete adjoint (with the
objective's explicit psi dependence) against complex-step directional
derivatives."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl

H_CS = 1e-30


def sw_particle(psi_value=1.0):
    """2x2 nodes, uniaxial anisotropy along y (B_K = 2K/Ms = 0.125 T), field
    ramped along x from 0 to B_K / 2 over 5 ns, strong damping."""
    K, Ms = 5e4, 8e5
    bk = 2 * K / Ms
    n, dt = 2500, 2e-12
    p = wl.Problem(nx=2, ny=2, nz=1, dx=3e-9, dy=3e-9, dz=3e-9, Ms=Ms, A=1.3e-11, K=K, ku=(0.0, 1.0, 0.0),
                   alpha0=1.0, alpha_max=1.0, b_rf=(0.5 * bk, 0.0, 0.0), drive_kind=1, t_ramp=n * dt,
                   terms=wl.TERM_EXCH | wl.TERM_ZEEMAN | wl.TERM_ANIS, dt=dt)
    m0 = np.zeros((3,) + p.shape)
    m0[1] = 1.0
    psi = np.full(p.shape, psi_value)
    return p, m0, psi, bk, n


def test_slow_ramp_follows_the_hard_axis_law():
    """A single-domain particle with its easy axis along y, field ramped slowly
    along x: M_x = B / B_K below saturation (Stoner-Wohlfarth hard axis).  The
    quasi-static lag of the damped response is below 1 % of B_K here."""
    p, m0, psi, bk, n = sw_particle()
    sim = mm.Sim(p, antenna=np.ones(p.shape))
    _, traj = sim.integrate(m0, psi, n, keep=True)
    obj = adj.Objective(adj.OBJ_MAG_CURVE, n_start=0, target=np.zeros(n), weight=np.ones(n))
    M = adj.curve_series(traj, psi, obj, n)
    B = 0.5 * bk * np.arange(1, n + 1) / n        # the ramp at t_n = n dt
    sel = slice(n // 2, n)                          # B from B_K / 4 to B_K / 2
    assert np.abs(M[sel] - B[sel] / bk).max() < 0.01
    assert M[-1] == pytest.approx(0.5, abs=0.01)


def test_curve_measure_is_the_particle_average():
    """M_x is the particle's average magnetisation: psi = 0.5 everywhere leaves
    the dynamics unchanged (Ms, A and K scale together) and leaves M_x
    unchanged too (a mean over the domain volume would halve it)."""
    p, m0, psi1, bk, n = sw_particle(1.0)
    _, _, psi2, _, _ = sw_particle(0.5)
    n = 200
    sim = mm.Sim(p, antenna=np.ones(p.shape))
    obj = adj.Objective(adj.OBJ_MAG_CURVE, n_start=0, target=np.zeros(n), weight=np.ones(n))
    M1 = adj.curve_series(sim.integrate(m0, psi1, n, keep=True)[1], psi1, obj, n)
    M2 = adj.curve_series(sim.integrate(m0, psi2, n, keep=True)[1], psi2, obj, n)
    assert np.abs(M1).max() > 0.02
    np.testing.assert_allclose(M2, M1, rtol=1e-12, atol=1e-15)


def test_curve_measure_of_a_binary_particle_is_the_mean_over_its_nodes():
    """psi = 1 on a few nodes and 0 elsewhere: M_x is the plain mean of m_x over
    those nodes, whatever the air nodes hold (brute force over the nodes)."""
    rng = np.random.default_rng(4)
    shape = (1, 5, 7)
    psi = np.zeros(shape)
    mag = [(0, 1, 2), (0, 1, 3), (0, 3, 5), (0, 4, 0)]
    for k in mag:
        psi[k] = 1.0
    traj = [rng.standard_normal((3,) + shape) for _ in range(4)]
    obj = adj.Objective(adj.OBJ_MAG_CURVE, n_start=1, target=np.zeros(2), weight=np.ones(2))
    M = adj.curve_series(traj, psi, obj, 3)
    want = [sum(traj[n][0][k] for k in mag) / len(mag) for n in (2, 3)]
    np.testing.assert_allclose(M, want, rtol=1e-14)
    # no material at all: M_x = 0
    assert np.all(adj.curve_series(traj, np.zeros(shape), obj, 3) == 0.0)


def test_paper_target_of_the_particle_workload():
    """The particle workload's target is M = 2 H_ext along the ramp 0 -> 0.3 Ms
    (0.6 n / N in units of Ms at step n of N) and its weights 1 / (M^target N)."""
    w = wl.sw_particle_curve(n_steps=400)
    tg, wt = w.extra["target"], w.extra["weight"]
    n = np.arange(1, 401)
    np.testing.assert_allclose(tg, 0.6 * n / 400, rtol=1e-15)
    np.testing.assert_allclose(wt, 1.0 / (tg * 400), rtol=1e-15)
    # the ramp itself reaches mu0 * 0.3 Ms along x at the last step
    assert w.problem.b_rf[0] == pytest.approx(4e-7 * np.pi * 0.3 * w.problem.Ms, rel=1e-15)
    assert w.problem.t_ramp == pytest.approx(400 * w.problem.dt, rel=1e-15)


def test_curve_adjoint_matches_complex_step():
    """dJ/dphi (through psi, including J's explicit psi dependence) and dJ/dm0
    against complex-step directional derivatives of the forward map."""
    p = wl.Problem(nx=6, ny=5, nz=1, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5, A=1.3e-11, K=2e4, ku=(0.0, 1.0, 0.0),
                   alpha0=0.5, alpha_max=0.5, b_rf=(0.08, 0.0, 0.0), drive_kind=1, t_ramp=30 * 5e-14,
                   terms=wl.TERM_ALL, dt=5e-14)
    rng = np.random.default_rng(9)
    sh = p.shape
    phi = rng.standard_normal((p.ny, p.nx)) * 0.5
    design = np.ones(sh)
    psif = np.zeros(sh)
    m0 = rng.standard_normal((3,) + sh) * 0.2
    m0[1] += 1.0
    m0 /= np.sqrt((m0 ** 2).sum(0))
    n, n_start = 30, 9
    W = n - n_start
    target = np.linspace(0.05, 0.3, W)
    obj = adj.Objective(adj.OBJ_MAG_CURVE, n_start=n_start, target=target, weight=1.0 / (target * W))
    sim = mm.Sim(p, antenna=np.ones(sh))
    a = 3.0
    psi = ls.levelset_to_psi(phi, a, design, psif)
    J, gpsi, lam0 = adj.gradient(sim, m0, psi, n, obj)
    gphi = ls.levelset_vjp(phi, a, design, gpsi)
    for _ in range(2):
        v = rng.standard_normal(phi.shape)
        Jc, _ = adj.forward_objective(sim, m0.astype(complex), ls.levelset_to_psi(phi + 1j * H_CS * v, a, design, psif),
                                      n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (gphi * v).sum()) <= 1e-11 * abs(d_cs)
        w = rng.standard_normal(m0.shape)
        Jc, _ = adj.forward_objective(sim, m0 + 1j * H_CS * w, psi.astype(complex), n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (lam0 * w).sum()) <= 1e-11 * abs(d_cs)
    assert abs(Jc.real - J) <= 1e-13 * abs(J)
