"""Pins of the oracle's size and centre constraints (Eq. 9): closed forms for a
uniform map and a single magnetic node, translation of the centre with the
material, and the gradient against complex steps and central differences."""
import numpy as np
import pytest

from oracle import shape

H_CS = 1e-30


def test_uniform_map_has_the_grid_centre_and_full_area():
    psi = np.full((2, 7, 10), 0.5)
    J = shape.penalty(psi, xi=1.0, S_target=0.0, nu=1.0, x0=0.0, y0=0.0)
    # S = 0.5 * 70, centre (4.5, 3)
    assert J == pytest.approx(35.0 ** 2 + 4.5 + 3.0, rel=1e-14)


def test_single_node_sits_at_its_own_coordinates():
    psi = np.zeros((1, 6, 8))
    psi[0, 4, 2] = 1.0
    assert shape.penalty(psi, xi=0.0, S_target=0.0, nu=1.0, x0=2.0, y0=4.0) == pytest.approx(0.0, abs=1e-15)
    assert shape.penalty(psi, xi=3.0, S_target=0.0, nu=0.0, x0=0.0, y0=0.0) == pytest.approx(3.0, rel=1e-15)


def test_shifting_the_material_shifts_the_centre():
    rng = np.random.default_rng(1)
    psi = np.zeros((1, 12, 15))
    psi[0, 2:7, 3:9] = rng.uniform(0.2, 1.0, (5, 6))
    shifted = np.roll(np.roll(psi, 3, axis=2), 4, axis=1)
    # with the targets moved by the same shift, the constraint is unchanged
    a = shape.penalty(psi, 0.7, 10.0, 2.0, 1.5, 2.5)
    b = shape.penalty(shifted, 0.7, 10.0, 2.0, 4.5, 6.5)
    assert a == pytest.approx(b, rel=1e-13)


def test_gradient_matches_complex_step_and_central_differences():
    rng = np.random.default_rng(2)
    psi = rng.uniform(0.05, 1.0, (2, 9, 11))
    args = (0.05, 40.0, 1.0, 3.2, 5.7)
    g = shape.penalty_grad(psi, *args)
    for _ in range(3):
        v = rng.standard_normal(psi.shape)
        d_cs = shape.penalty(psi + 1j * H_CS * v, *args).imag / H_CS
        assert abs(d_cs - (g * v).sum()) <= 1e-12 * abs(d_cs)
        h = 1e-6
        d_fd = (shape.penalty(psi + h * v, *args) - shape.penalty(psi - h * v, *args)) / (2 * h)
        assert abs(d_fd - (g * v).sum()) <= 1e-6 * abs(d_fd)
