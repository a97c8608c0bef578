"""Pins of the oracle's demagnetisation tensor and demag convolution.

Each expected value comes from mathematics independent of the oracle code:
Aharoni's closed-form prism factors, the trace identity of the demag tensor,
its parities, the point-dipole far field, and the O(N^2) direct sum.
"""
import math

import numpy as np
import pytest

from oracle import micromag as mm
from oracle import newell as nw


def aharoni_nzz(a, b, c):
    """Demagnetising factor along z of a 2a x 2b x 2c prism (A. Aharoni,
    J. Appl. Phys. 83, 3432 (1998), Eq. 1)."""
    r = math.sqrt(a * a + b * b + c * c)
    ab, bc, ac = math.hypot(a, b), math.hypot(b, c), math.hypot(a, c)
    s = ((b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
         + b / (2 * c) * math.log((ab + a) / (ab - a))
         + a / (2 * c) * math.log((ab + b) / (ab - b))
         + c / (2 * a) * math.log((bc - b) / (bc + b))
         + c / (2 * b) * math.log((ac - a) / (ac + a))
         + 2 * math.atan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / math.pi


CELLS = [(1.0, 1.0, 1.0), (5e-9, 5e-9, 10e-9), (2.0, 3.0, 1.0), (4e-9, 4e-9, 5e-9), (1.0, 10.0, 1.0), (3.0, 1.0, 0.2)]


def _self(h):
    z = np.zeros(1)
    return nw.tensor_at(z, z, z, h)[:, 0]


@pytest.mark.parametrize("h", CELLS)
def test_self_term_matches_aharoni_all_axes(h):
    N0 = _self(h)
    hx, hy, hz = h
    # the z-factor of the prism, and the x/y factors by relabelling the axes
    assert abs(N0[2] - aharoni_nzz(hx / 2, hy / 2, hz / 2)) < 1e-13
    assert abs(N0[0] - aharoni_nzz(hy / 2, hz / 2, hx / 2)) < 1e-13
    assert abs(N0[1] - aharoni_nzz(hz / 2, hx / 2, hy / 2)) < 1e-13
    assert abs(N0[:3].sum() - 1.0) < 1e-14
    assert np.all(np.abs(N0[3:]) < 1e-15)


def test_cube_self_term_is_one_third():
    N0 = _self((2e-9, 2e-9, 2e-9))
    assert np.allclose(N0[:3], 1.0 / 3.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("h", [(5e-9, 5e-9, 10e-9), (2.0, 3.0, 1.0)])
def test_trace_vanishes_off_origin_and_parities(h):
    rng = np.random.default_rng(0)
    offs = rng.integers(-12, 13, size=(60, 3)).astype(float)
    offs = offs[np.abs(offs).sum(1) > 0]
    X, Y, Z = offs[:, 0] * h[0], offs[:, 1] * h[1], offs[:, 2] * h[2]
    N = nw.tensor_at(X, Y, Z, h)
    scale = np.abs(N).max(axis=0)
    assert np.all(np.abs(N[:3].sum(0)) <= 1e-11 * scale + 1e-300)
    for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
        Nm = nw.tensor_at(sx * X, sy * Y, sz * Z, h)
        for c in range(6):
            par = nw.PARITY[c]
            sign = (par[0] if sx < 0 else 1) * (par[1] if sy < 0 else 1) * (par[2] if sz < 0 else 1)
            assert np.allclose(Nm[c], sign * N[c], rtol=1e-12, atol=1e-12 * scale.max())


def test_far_field_tends_to_point_dipole():
    h = (5e-9, 5e-9, 10e-9)
    V = h[0] * h[1] * h[2]
    for d in (np.array([1.0, 0.3, 0.2]), np.array([0.2, 1.0, 0.5])):
        errs = []
        for R in (40e-9, 80e-9, 160e-9):
            r = d / np.linalg.norm(d) * R
            N = nw.tensor_at(np.array([r[0]]), np.array([r[1]]), np.array([r[2]]), h)[:, 0]
            rh = r / R
            D = -(3 * np.outer(rh, rh) - np.eye(3)) / (4 * math.pi * R ** 3) * V
            ref = np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])
            errs.append(np.abs(N - ref).max() / np.abs(ref).max())
        # quadrupole-free: the relative deviation falls like (h/R)^2
        assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0
        assert errs[2] < 5e-3


def test_closed_form_agrees_with_converged_quadrature():
    """For separated cells the integral definition converges under high-order
    Gauss-Legendre; the Newell closed form must agree with it."""
    for h in [(5e-9, 5e-9, 10e-9), (1.0, 1.0, 1.0), (2.0, 3.0, 1.0)]:
        for off in [(2, 0, 0), (2, 1, 0), (3, 2, 1), (0, 2, 2), (4, 1, 0)]:
            r = [np.array([off[i] * h[i]]) for i in range(3)]
            ex = nw.newell_exact(*r, h)[:, 0]
            q = nw.dipole_quadrature(*r, h, 24)[:, 0]
            assert np.abs(ex - q).max() <= 1e-11 * np.abs(q).max()


def test_near_far_switch_is_continuous():
    """Both evaluation methods on either side of the switch agree."""
    h = (4e-9, 4e-9, 5e-9)
    for off in [(3, 0, 0), (3, 2, 0), (2, 2, 1), (0, 3, 1)]:
        r = [np.array([off[i] * h[i]]) for i in range(3)]
        ex = nw.newell_exact(*r, h)[:, 0]
        q8 = nw.dipole_quadrature(*r, h, 8)[:, 0]
        assert np.abs(ex - q8).max() <= 1e-10 * np.abs(ex).max()


@pytest.mark.parametrize("shape,h", [((3, 4, 5), (3e-9, 4e-9, 5e-9)), ((1, 5, 7), (5e-9, 5e-9, 10e-9)),
                                     ((2, 1, 6), (2e-9, 2e-9, 3e-9))])
def test_fft_convolution_equals_direct_sum(shape, h):
    nz, ny, nx = shape
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3,) + shape)
    K = mm.DemagKernel(nx, ny, nz, h)
    a = K.conv(x)
    b = mm.demag_direct(x, h)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    # any padding >= 2n - 1 gives the same linear convolution
    P2 = tuple(1 if n == 1 else 2 * n + 3 for n in shape)
    c = mm.DemagKernel(nx, ny, nz, h, pad=P2).conv(x)
    assert np.abs(a - c).max() <= 1e-13 * np.abs(b).max()
