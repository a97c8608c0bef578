"""Pins of the oracle's discrete adjoint and level-set map.

The adjoint (hand-derived transposes of every field term and of the RK4 step)
is checked against derivatives of the *forward* map taken independently of
it: complex-step directional derivatives (exact to rounding, no subtractive
cancellation) and central finite differences.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl

H_CS = 1e-30


def tiny_problem(terms=wl.TERM_ALL):
    return wl.Problem(nx=7, ny=5, nz=2, dx=3e-9, dy=3e-9, dz=4e-9, Ms=8e5, A=1.3e-11, K=5e4, ku=(0.6, 0.8, 0.0),
                      alpha0=0.1, alpha_max=0.4, ramp_cells=3, ramp_faces=wl.FACE_XLO | wl.FACE_XHI,
                      B0=(0.05, 0.02, 0.1), b_rf=(0.0, 0.01, 0.0), f1=5e9, terms=terms, dt=5e-14)


def tiny_inputs(p, seed=5):
    rng = np.random.default_rng(seed)
    sh = p.shape
    ant = np.zeros(sh)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((p.ny, p.nx)) * 0.5
    design = np.ones(sh)
    design[:, 0, :] = 0
    psif = np.full(sh, 0.7)
    psif[:, 0, :3] = 0.0             # frozen air nodes outside the design region
    m0 = rng.standard_normal((3,) + sh)
    m0 /= np.sqrt((m0 ** 2).sum(0))
    p1 = np.zeros(sh)
    p1[:, 3:, 4:] = 1
    p2 = np.zeros(sh)
    p2[:, 1:3, 4:] = 1
    return ant, phi, design, psif, m0, p1, p2


@pytest.mark.parametrize("kind", [adj.OBJ_ENERGY_AREA, adj.OBJ_PORT_MY2])
@pytest.mark.parametrize("terms", [wl.TERM_ALL, wl.TERM_EXCH | wl.TERM_ZEEMAN])
def test_adjoint_gradient_matches_complex_step(kind, terms):
    p = tiny_problem(terms)
    ant, phi, design, psif, m0, p1, p2 = tiny_inputs(p)
    sim = mm.Sim(p, antenna=ant)
    a = 3.0
    obj = adj.Objective(kind, E_ref=1e-18, lam=0.7, area=0.4, n_start=10, port1=p1, port2=p2)
    n = 25
    psi = ls.levelset_to_psi(phi, a, design, psif)
    J, gpsi, lam0 = adj.gradient(sim, m0, psi, n, obj)
    gphi = ls.levelset_vjp(phi, a, design, gpsi)
    rng = np.random.default_rng(11)
    for _ in range(2):
        v = rng.standard_normal(phi.shape)
        Jc, _ = adj.forward_objective(sim, m0.astype(complex), ls.levelset_to_psi(phi + 1j * H_CS * v, a, design, psif), n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (gphi * v).sum()) <= 1e-12 * abs(d_cs)
        w = rng.standard_normal(m0.shape)
        Jc, _ = adj.forward_objective(sim, m0 + 1j * H_CS * w, psi.astype(complex), n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (lam0 * w).sum()) <= 1e-12 * abs(d_cs)
    assert abs(Jc.real - J) <= 1e-14 * abs(J)


def test_rhs_transpose_dot_product():
    """<J_f v, w> = <v, J_f^T w> and <df/dpsi q, w> = <q, g> for one RHS evaluation."""
    p = tiny_problem()
    ant, phi, design, psif, m0, _, _ = tiny_inputs(p)
    sim = mm.Sim(p, antenna=ant)
    psi = ls.levelset_to_psi(phi, 3.0, design, psif)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(m0.shape)
    q = rng.standard_normal(psi.shape) * (psi != 0)
    w = rng.standard_normal(m0.shape)
    t = 3.3e-11
    f_m, _ = sim.rhs(m0 + 1j * H_CS * v, psi.astype(complex), t)
    f_p, _ = sim.rhs(m0.astype(complex), psi + 1j * H_CS * q, t)
    _, B = sim.rhs(m0, psi, t)
    mu, g = adj.rhs_vjp(sim, m0, B, psi, w)
    lhs_m = ((f_m.imag / H_CS) * w).sum()
    lhs_p = ((f_p.imag / H_CS) * w).sum()
    assert abs(lhs_m - (v * mu).sum()) <= 1e-13 * np.abs(f_m.imag / H_CS).max() * np.abs(w).sum()
    assert abs(lhs_p - (q * g).sum()) <= 1e-13 * np.abs(f_p.imag / H_CS).max() * np.abs(w).sum()


def test_energy_objective_gradient_central_fd():
    """Permalloy-particle objective on a reduced grid: adjoint vs central FD at
    seeded random nodes (FD truncation ~delta^2, rounding ~eps/delta)."""
    w = wl.permalloy_particle(nx=12, ny=10, n_steps=60)
    p = w.problem
    sim = mm.Sim(p)
    obj = adj.Objective(adj.OBJ_ENERGY_AREA, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area)
    psi = ls.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    J, gpsi, _ = adj.gradient(sim, w.m0, psi, w.n_steps, obj)
    gphi = ls.levelset_vjp(w.phi, w.heaviside_a, w.design, gpsi)
    rng = np.random.default_rng(0)
    for node in rng.choice(w.phi.size, 4, replace=False):
        iy, ix = divmod(int(node), p.nx)
        d = 1e-5 * max(1.0, abs(w.phi[iy, ix]))
        Js = []
        for s in (1, -1):
            ph = w.phi.copy()
            ph[iy, ix] += s * d
            Js.append(adj.forward_objective(sim, w.m0, ls.levelset_to_psi(ph, w.heaviside_a, w.design, w.psi_fixed),
                                            w.n_steps, obj)[0])
        fd = (Js[0] - Js[1]) / (2 * d)
        assert abs(fd - gphi[iy, ix]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gphi).max())


def test_heaviside_identities():
    phi = np.linspace(-3, 3, 101)
    for a in (4.0 / 3.0, 20.0, 50.0):
        H = ls.heaviside(phi, a)
        assert abs(ls.heaviside(np.array(0.0), a) - 0.5) < 1e-16
        assert np.allclose(ls.heaviside(-phi, a), 1.0 - H, rtol=0, atol=1e-15)
        assert np.allclose(H, 0.5 * (1.0 + np.tanh(0.5 * a * phi)), rtol=0, atol=1e-15)
        assert np.all(H > 0)
        hp = ls.heaviside_prime(phi, a)
        fd = (ls.heaviside(phi + 1e-6, a) - ls.heaviside(phi - 1e-6, a)) / 2e-6
        assert np.allclose(hp, fd, rtol=1e-6, atol=1e-8)


def test_levelset_extrusion_vjp_sums_over_thickness():
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((5, 6))
    design = np.ones((3, 5, 6))
    design[:, :, 0] = 0
    g = rng.standard_normal((3, 5, 6))
    gphi = ls.levelset_vjp(phi, 2.0, design, g)
    q = rng.standard_normal(phi.shape)
    psic = ls.levelset_to_psi(phi + 1j * H_CS * q, 2.0, design, np.zeros((3, 5, 6)))
    assert abs((psic.imag / H_CS * g).sum() - (gphi * q).sum()) < 1e-13 * np.abs(g).sum()
    assert np.all(gphi[:, 0] == 0)


def test_workload_layouts_are_consistent():
    w = wl.yig_demux(n_steps=10)
    assert w.phi.shape == (96, 256)
    assert np.all(w.phi[w.design[0] == 0] == 0)
    assert abs(np.abs(w.phi).max() - 1.0) < 1e-15
    for mk in (w.antenna, w.port1, w.port2):
        assert mk.sum() > 0
        assert np.all(w.psi_fixed[mk.astype(bool)] == 1.0)
    assert not np.any(w.port1 & w.port2)
    ws = wl.yig_demux_sweep(n_steps=10)
    assert len(ws) == 64
    for w in ws:
        assert 128 <= w.problem.nx <= 256 and 64 <= w.problem.ny <= 128
