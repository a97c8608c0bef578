"""Pins of the oracle's continuous adjoint (Eqs. 6-7 integrated backwards):
it approaches the discrete adjoint at fourth order as the steps shrink, on
fixed and on adaptive step sequences, with and without sub-steps; on a stiff
adaptive run one RK4 step per interval diverges and two do not; the Hermite
interpolant reproduces cubics exactly."""
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


def both(sim, m0, psi, obj, hs, n_sub=1):
    Jd, gd, ld = dopri.gradient_fixed(sim, m0, psi, 0.0, hs, obj)
    mT, traj = dopri.integrate_fixed(sim, m0, psi, 0.0, hs, keep=True)
    ts = [0.0]
    for h in hs:
        ts.append(ts[-1] + h)
    lamT, gT = adj.energy_area_grad(sim, mT, psi, obj)
    gc, lc = cont.continuous_adjoint(sim, traj, ts, hs, psi, lamT, gT, n_sub=n_sub)
    return gd, ld, gc, lc


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n_sub", [1, 2])
def test_continuous_adjoint_approaches_the_discrete_one_at_fourth_order(n_sub):
    sim, m0, psi, obj = setup()
    T = 4e-12
    d = []
    for n in (40, 80):
        gd, ld, gc, lc = both(sim, m0, psi, obj, [T / n] * n, n_sub=n_sub)
        d.append((rel(gc, gd), rel(lc, ld)))
    assert d[1][0] < 1e-5 and d[1][1] < 1e-5
    for k in (0, 1):
        assert 10.0 < d[0][k] / d[1][k] < 40.0


def test_continuous_adjoint_on_adaptive_steps():
    sim, m0, psi, obj = setup(seed=15)
    _, hs, _ = dopri.integrate_adaptive(sim, m0, psi, 0.0, 4e-12, 5e-14, rtol=1e-8, atol=1e-8)
    gd, ld, gc, lc = both(sim, m0, psi, obj, hs)
    assert rel(gc, gd) < 1e-3 and rel(lc, ld) < 1e-3


def test_hermite_interpolant_is_exact_for_cubics():
    """A cubic x(t) with its end values and slopes is reproduced at any th."""
    c = np.array([0.3, -1.2, 0.7, 2.5])
    x = lambda s: c[0] + c[1] * s + c[2] * s ** 2 + c[3] * s ** 3
    dx = lambda s: c[1] + 2 * c[2] * s + 3 * c[3] * s ** 2
    t0, h = 0.4, 0.9
    for th in (0.0, 0.25, 0.5, 0.8, 1.0):
        assert cont.hermite(x(t0), x(t0 + h), dx(t0), dx(t0 + h), h, th) == pytest.approx(x(t0 + th * h), abs=1e-14)


def test_sub_steps_keep_the_backward_pass_stable_on_a_stiff_adaptive_run():
    """Permalloy particle, 12x10 nodes of 2 nm: the adaptive run's steps sit at
    the edge of Dormand-Prince's stability region, beyond RK4's, so the
    backward pass with one RK4 step per interval diverges; with two sub-steps
    it agrees with the discrete adjoint."""
    w = wl.permalloy_particle(nx=12, ny=10, n_steps=400)
    p = w.problem
    sim = mm.Sim(p)
    psi = ls.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    obj = adj.Objective(w.objective, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area)
    _, hs, rej = dopri.integrate_adaptive(sim, w.m0, psi, 0.0, w.n_steps * p.dt, p.dt, 1e-5, 1e-5)
    assert rej > 0
    gd, ld, gc1, lc1 = both(sim, w.m0, psi, obj, hs, n_sub=1)
    assert rel(gc1, gd) > 1e3 and rel(lc1, ld) > 1e3
    _, _, gc2, lc2 = both(sim, w.m0, psi, obj, hs, n_sub=2)
    assert rel(gc2, gd) < 1e-4 and rel(lc2, ld) < 1e-3
