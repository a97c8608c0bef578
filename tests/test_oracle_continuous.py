"""Pins of the oracle's continuous adjoint (Eqs. 6-7 integrated backwards):
it approaches the discrete adjoint at fourth order as the steps shrink, on
fixed and on adaptive step sequences."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import continuous as cont
from oracle import dopri
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl


def setup(seed=14):
    p = wl.Problem(nx=6, ny=5, nz=1, dx=3e-9, dy=3e-9, dz=4e-9, Ms=8e5, A=1.3e-11, K=5e4, ku=(0.6, 0.8, 0.0),
                   alpha0=0.2, alpha_max=0.2, B0=(0.05, 0.02, 0.1), b_rf=(0.0, 0.01, 0.0), f1=5e9,
                   terms=wl.TERM_ALL, dt=5e-14)
    rng = np.random.default_rng(seed)
    sh = p.shape
    ant = np.zeros(sh)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((p.ny, p.nx)) * 0.5
    m0 = rng.standard_normal((3,) + sh)
    m0 /= np.sqrt((m0 ** 2).sum(0))
    sim = mm.Sim(p, antenna=ant)
    psi = ls.levelset_to_psi(phi, 3.0, np.ones(sh), np.zeros(sh))
    obj = adj.Objective(adj.OBJ_ENERGY_AREA, E_ref=1e-18, lam=0.7, area=0.4)
    return sim, m0, psi, obj


def both(sim, m0, psi, obj, hs):
    Jd, gd, ld = dopri.gradient_fixed(sim, m0, psi, 0.0, hs, obj)
    mT, traj = dopri.integrate_fixed(sim, m0, psi, 0.0, hs, keep=True)
    ts = [0.0]
    for h in hs:
        ts.append(ts[-1] + h)
    lamT, gT = adj.energy_area_grad(sim, mT, psi, obj)
    gc, lc = cont.continuous_adjoint(sim, traj, ts, hs, psi, lamT, gT)
    return gd, ld, gc, lc


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_continuous_adjoint_approaches_the_discrete_one_at_fourth_order():
    sim, m0, psi, obj = setup()
    T = 4e-12
    d = []
    for n in (40, 80):
        gd, ld, gc, lc = both(sim, m0, psi, obj, [T / n] * n)
        d.append((rel(gc, gd), rel(lc, ld)))
    assert d[1][0] < 1e-5 and d[1][1] < 1e-5
    for k in (0, 1):
        assert 10.0 < d[0][k] / d[1][k] < 40.0


def test_continuous_adjoint_on_adaptive_steps():
    sim, m0, psi, obj = setup(seed=15)
    _, hs, _ = dopri.integrate_adaptive(sim, m0, psi, 0.0, 4e-12, 5e-14, rtol=1e-8, atol=1e-8)
    gd, ld, gc, lc = both(sim, m0, psi, obj, hs)
    assert rel(gc, gd) < 1e-3 and rel(lc, ld) < 1e-3
