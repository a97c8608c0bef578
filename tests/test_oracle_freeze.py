"""Pins of the oracle's frozen-node threshold (psi_freeze, an option beyond the
paper): nodes with psi <= psi_freeze keep their state exactly while the rest
move; a threshold of 0 is the method as stated (only psi = 0 frozen); and the
discrete adjoint stays the exact gradient of the modified map, checked against
complex-step directional derivatives in phi and m0 (the frozen set is decided
on the real part of psi, so a complex step does not move it)."""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl

H_CS = 1e-30


def setup(freeze):
    p = wl.Problem(nx=9, ny=7, nz=1, dx=5e-9, dy=5e-9, dz=10e-9, Ms=1.4e5, A=3.5e-12, alpha0=1e-2, alpha_max=0.2,
                   ramp_cells=2, ramp_faces=wl.FACE_XLO | wl.FACE_XHI, B0=(0.0, 0.0, 0.2), b_rf=(0.0, 5e-3, 0.0),
                   f1=3e9, terms=wl.TERM_ALL, dt=1e-13, psi_freeze=freeze)
    rng = np.random.default_rng(7)
    sh = p.shape
    ant = np.zeros(sh)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((p.ny, p.nx)) * 0.2
    design = np.ones(sh)
    design[:, :, :2] = 0
    psif = np.where(np.arange(p.nx)[None, None, :] < 2, 1.0, 0.0) * np.ones(sh)
    m0 = rng.standard_normal((3,) + sh) * 0.1
    m0[2] += 1.0
    m0 /= np.sqrt((m0 ** 2).sum(0))
    p1 = np.zeros(sh)
    p1[:, 4:, 6:] = 1
    p2 = np.zeros(sh)
    p2[:, :3, 6:] = 1
    return p, ant, phi, design, psif, m0, p1, p2


A_LS = 30.0


def test_frozen_nodes_keep_their_state():
    p, ant, phi, design, psif, m0, _, _ = setup(0.05)
    psi = ls.levelset_to_psi(phi, A_LS, design, psif)
    frozen = psi <= 0.05
    assert 0 < frozen.sum() < frozen.size and (frozen & (psi > 0)).any()
    mT = mm.Sim(p, antenna=ant).integrate(m0, psi, 20)
    assert np.array_equal(mT[:, frozen], m0[:, frozen])
    assert np.abs(mT[:, ~frozen] - m0[:, ~frozen]).max() > 1e-6


def test_zero_threshold_is_the_method_as_stated():
    p0, ant, phi, design, psif, m0, _, _ = setup(0.0)
    p_default = dataclasses.replace(p0)
    del p_default.psi_freeze  # an object without the attribute: the default rule
    psi = ls.levelset_to_psi(phi, A_LS, design, psif)
    a = mm.Sim(p0, antenna=ant).integrate(m0, psi, 15)
    b = mm.Sim(p_default, antenna=ant).integrate(m0, psi, 15)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("freeze", [0.05, 1e-3])
def test_frozen_map_adjoint_matches_complex_step(freeze):
    p, ant, phi, design, psif, m0, p1, p2 = setup(freeze)
    sim = mm.Sim(p, antenna=ant)
    n = 30
    obj = adj.Objective(adj.OBJ_PORT_MY2, n_start=10, port1=p1, port2=p2)
    psi = ls.levelset_to_psi(phi, A_LS, design, psif)
    assert (psi <= freeze).any()
    J, gpsi, lam0 = adj.gradient(sim, m0, psi, n, obj)
    gphi = ls.levelset_vjp(phi, A_LS, design, gpsi)
    rng = np.random.default_rng(12)
    for _ in range(2):
        v = rng.standard_normal(phi.shape)
        Jc, _ = adj.forward_objective(sim, m0.astype(complex), ls.levelset_to_psi(phi + 1j * H_CS * v, A_LS, design, psif),
                                      n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (gphi * v).sum()) <= 1e-11 * abs(d_cs)
        w = rng.standard_normal(m0.shape)
        Jc, _ = adj.forward_objective(sim, m0 + 1j * H_CS * w, psi.astype(complex), n, obj)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (lam0 * w).sum()) <= 1e-11 * abs(d_cs)
