"""Size and centre-of-mass constraints of the regularised objective (Eq. 9).

Oracle (test infrastructure only).

Eq. 9 adds to the magnetisation-curve term a size constraint xi (S - S_t)^2 and
a centre constraint nu (|x_c - x_0| + |y_c - y_0|), with S the particle's area
and (x_c, y_c) its centre of mass.  Readings: S = sum_i psi_i / nz (the
in-plane area in cells of the material map, averaged over the layers); x_c =
sum_i psi_i x_i / sum_i psi_i and y_c likewise, with x_i, y_i node indices;
|.| takes the zero subgradient at 0.  The terms depend on psi only, so their
gradient enters the adjoint as an explicit dJ/dpsi.
"""
from __future__ import annotations

import numpy as np


def _absr(z):
    return np.where(np.real(z) >= 0, z, -z)


def penalty(psi, xi, S_target, nu, x0, y0):
    """J of the two constraints for psi of shape (nz, ny, nx)."""
    nz, ny, nx = psi.shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tot = psi.sum()
    S = tot / nz
    xc = (psi * X).sum() / tot
    yc = (psi * Y).sum() / tot
    return xi * (S - S_target) ** 2 + nu * (_absr(xc - x0) + _absr(yc - y0))


def penalty_grad(psi, xi, S_target, nu, x0, y0):
    """dJ/dpsi: 2 xi (S - S_t) / nz + nu [sgn(x_c - x0)(x_i - x_c) + sgn(y_c - y0)(y_i - y_c)] / sum psi."""
    nz, ny, nx = psi.shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tot = psi.sum()
    S = tot / nz
    xc = (psi * X).sum() / tot
    yc = (psi * Y).sum() / tot
    return (2.0 * xi * (S - S_target) / nz
            + nu * (np.sign(xc - x0) * (X - xc) + np.sign(yc - y0) * (Y - yc)) / tot)
