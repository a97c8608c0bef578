"""Pins of the oracle's spectral port objective (Eq. 10) and the two-tone
drive: DFT magnitudes of sinusoids over whole periods, orthogonality of the
DFT bins, positive homogeneity, derivatives against complex steps, and the
discrete adjoint of the full forward map against complex-step directional
derivatives."""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import levelset as ls
from oracle import micromag as mm
from paper_2411_19109_amd import workloads as wl

H_CS = 1e-30


def obj_with(freqs, coef, n_start=0, port1=None, port2=None):
    return adj.Objective(adj.OBJ_PORT_SPECTRAL, n_start=n_start, port1=port1, port2=port2, freqs=freqs, coef=coef)


def test_dft_of_a_sinusoid_over_whole_periods():
    """x(n) = A cos(2 pi f t_n + phase) over W samples spanning whole periods
    (W f dt and 2 W f dt integers): |X(f)| = A/2, and |X| vanishes at the other
    DFT bins f + k / (W dt)."""
    dt, W = 1e-13, 400
    times = np.arange(1, W + 1) * dt
    f = 25 / (W * dt)                       # 25 whole periods
    A, ph = 0.37, 0.8
    x = np.array([A * np.cos(2 * np.pi * f * times + ph), -2.0 * np.cos(2 * np.pi * f * times)])
    bins = np.array([f, f + 3 / (W * dt), f - 7 / (W * dt)])
    C, S = adj.spectral_parts(x, times, bins)
    mag = np.sqrt(C * C + S * S)
    assert mag[0, 0] == pytest.approx(A / 2, rel=1e-12)
    assert mag[1, 0] == pytest.approx(1.0, rel=1e-12)
    assert np.abs(mag[:, 1:]).max() < 1e-14
    # the phase: X = A/2 exp(i phase) at the positive frequency (X = C - i S)
    assert math.atan2(-S[0, 0], C[0, 0]) == pytest.approx(ph, abs=1e-12)


def test_two_tone_drive_has_half_unit_lines_at_both_frequencies():
    """Without a switch and with f2 > 0 the drive is the sum of two unit sines:
    its DFT over whole periods of both has magnitude 1/2 at f1 and at f2."""
    dt, W = 1e-13, 1000
    f1, f2 = 26 / (W * dt), 28 / (W * dt)    # 2.6 and 2.8 GHz, the paper's demultiplexer pair
    p = wl.Problem(nx=2, ny=2, nz=1, dx=5e-9, dy=5e-9, dz=10e-9, Ms=1.4e5, A=3.5e-12, f1=f1, f2=f2, dt=dt)
    sim = mm.Sim(p)
    times = np.arange(1, W + 1) * dt
    x = np.array([[sim.drive(t) for t in times], [0.0] * W])
    C, S = adj.spectral_parts(x, times, np.array([f1, f2, 27 / (W * dt)]))
    mag = np.sqrt(C * C + S * S)[0]
    np.testing.assert_allclose(mag, [0.5, 0.5, 0.0], atol=1e-13)
    # a switch time keeps the single-frequency-then-switch behaviour
    p.t_switch = 5e-11
    assert sim.drive(1e-11) == pytest.approx(math.sin(2 * math.pi * f1 * 1e-11), abs=1e-15)


def test_spectral_objective_is_positively_homogeneous_and_its_sources_match_complex_step():
    rng = np.random.default_rng(3)
    dt, W = 1e-13, 300
    times = 5e-12 + np.arange(W) * dt
    freqs = np.array([2.4e9, 2.5e9, 2.6e9, 3.4e9, 3.5e9, 3.6e9])
    coef = np.array([[1, 1, 1, -1, -1, -1], [-1, -1, -1, 1, 1, 1]], float)
    obj = obj_with(freqs, coef)
    x = rng.standard_normal((2, W)) * 1e-3
    J = adj.spectral_value(x, times, obj)
    assert adj.spectral_value(-2.5 * x, times, obj) == pytest.approx(2.5 * J, rel=1e-13)
    g = adj.spectral_sources(x, times, obj)
    for _ in range(3):
        v = rng.standard_normal((2, W))
        d_cs = adj.spectral_value(x + 1j * H_CS * v, times, obj).imag / H_CS
        assert abs(d_cs - (g * v).sum()) <= 1e-12 * abs(d_cs)


def tiny_two_tone():
    p = wl.Problem(nx=7, ny=5, nz=2, dx=3e-9, dy=3e-9, dz=4e-9, Ms=8e5, A=1.3e-11, K=5e4, ku=(0.6, 0.8, 0.0),
                   alpha0=0.1, alpha_max=0.4, ramp_cells=3, ramp_faces=wl.FACE_XLO | wl.FACE_XHI,
                   B0=(0.05, 0.02, 0.1), b_rf=(0.0, 0.01, 0.0), f1=5e9, f2=8e9, terms=wl.TERM_ALL, dt=5e-14)
    rng = np.random.default_rng(5)
    sh = p.shape
    ant = np.zeros(sh)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((p.ny, p.nx)) * 0.5
    design = np.ones(sh)
    design[:, 0, :] = 0
    psif = np.full(sh, 0.7)
    m0 = rng.standard_normal((3,) + sh)
    m0 /= np.sqrt((m0 ** 2).sum(0))
    p1 = np.zeros(sh)
    p1[:, 3:, 4:] = 1
    p2 = np.zeros(sh)
    p2[:, 1:3, 4:] = 1
    return p, ant, phi, design, psif, m0, p1, p2


@pytest.mark.parametrize("t0", [0.0, 3e-12])
def test_spectral_adjoint_gradient_matches_complex_step(t0):
    """dJ/dphi and dJ/dm0 of the spectral objective by the discrete adjoint
    against complex-step directional derivatives of the forward map."""
    p, ant, phi, design, psif, m0, p1, p2 = tiny_two_tone()
    sim = mm.Sim(p, antenna=ant)
    a = 3.0
    freqs = np.array([4.5e9, 5e9, 5.5e9, 7.5e9, 8e9, 8.5e9])
    coef = np.array([[1, 1, 1, -1, -1, -1], [-1, -1, -1, 1, 1, 1]], float)
    obj = obj_with(freqs, coef, n_start=8, port1=p1, port2=p2)
    n = 24
    psi = ls.levelset_to_psi(phi, a, design, psif)
    J, gpsi, lam0 = adj.gradient(sim, m0, psi, n, obj, t0=t0)
    gphi = ls.levelset_vjp(phi, a, design, gpsi)
    rng = np.random.default_rng(11)
    for _ in range(2):
        v = rng.standard_normal(phi.shape)
        Jc, _ = adj.forward_objective(sim, m0.astype(complex), ls.levelset_to_psi(phi + 1j * H_CS * v, a, design, psif),
                                      n, obj, t0=t0)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (gphi * v).sum()) <= 1e-11 * abs(d_cs)
        w = rng.standard_normal(m0.shape)
        Jc, _ = adj.forward_objective(sim, m0 + 1j * H_CS * w, psi.astype(complex), n, obj, t0=t0)
        d_cs = Jc.imag / H_CS
        assert abs(d_cs - (lam0 * w).sum()) <= 1e-11 * abs(d_cs)
    # J is a difference of window sums that nearly cancel here: compare on their scale
    assert abs(Jc.real - J) <= 1e-13 * np.abs(obj.coef).sum() * np.abs(adj.port_series(
        mm.Sim(p, antenna=ant).integrate(m0, psi, n, t0=t0, keep=True)[1], obj, n)).max()
