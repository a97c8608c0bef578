"""Level-set to material map (Eq. 4 and the paragraph after it).

Oracle (test infrastructure only).

psi = D * H(phi) + (1 - D) * psi_fixed, with the smoothed Heaviside
H(phi) = 1 / (1 + exp(-a phi)) (the paper's sigmoid, Eq. 4), evaluated in
exactly that form: it tends to 0 gracefully for a*phi -> -inf, whereas the
equivalent (1 + tanh(a phi / 2)) / 2 rounds to exactly 0 once tanh rounds to
-1 (a*phi < -38 in float64).  D marks the design
region (1 inside, 0 outside); psi_fixed describes the fixed geometry outside
it.  A two-dimensional phi can be extruded through the film thickness.
"""
from __future__ import annotations

import numpy as np


def heaviside(phi, a):
    return 1.0 / (1.0 + np.exp(-a * phi))


def heaviside_prime(phi, a):
    H = heaviside(phi, a)
    return a * H * (1.0 - H)


def levelset_to_psi(phi, a, design, psi_fixed, nz=None):
    """psi (nz, ny, nx) from phi of shape (ny, nx) (extruded) or (nz, ny, nx)."""
    D = np.asarray(design, float)
    if phi.ndim == 2:
        phi = np.broadcast_to(phi, D.shape)
    return D * heaviside(phi, a) + (1.0 - D) * np.asarray(psi_fixed, float)


def levelset_vjp(phi, a, design, g_psi):
    """dJ/dphi = D * H'(phi) * dJ/dpsi, summed over z when phi is extruded."""
    D = np.asarray(design, float)
    if phi.ndim == 2:
        return (D * heaviside_prime(np.broadcast_to(phi, D.shape), a) * g_psi).sum(axis=0)
    return D * heaviside_prime(phi, a) * g_psi
