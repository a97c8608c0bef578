"""Level-set function from radial basis functions (Eqs. 2 and 3) and the Adam
update of their amplitudes.

Oracle (test infrastructure only).

Eq. 2: each RBF is a multiquadric cone g_i(x, y) = s_i - sqrt((x - x_i)^2 +
(y - y_i)^2 + c^2) with amplitude s_i.  Eq. 3: the level-set function is the
p-norm soft maximum of the cones, shifted by dphi so that the bases are
non-negative,

    Phi(x, y) = [ sum_i (g_i(x, y) + dphi)^p ]^(1/p) - dphi,

with dphi the absolute value of the smallest cone value on the design region.
The paper keeps Phi in [-1, 1] by renormalising it; here that is a division by
max |Phi| over the design region.  Readings: coordinates are node indices
(x = ix, y = iy), c in the same units; dphi and the renormalisation factor are
recomputed from the current amplitudes on every evaluation and held fixed in
the derivative (the shift and the scale are chosen, not differentiated); a
node whose bases are all 0 (the p-norm's kink, possible when one cone is the
only one that reaches the shift's node) takes the zero subgradient.

The Adam update follows Kingma & Ba (2015), Algorithm 1, bias-corrected.
"""
from __future__ import annotations

import numpy as np


def cones(s, centers, c, nx, ny):
    """g[i, iy, ix] = s_i - sqrt((ix - x_i)^2 + (iy - y_i)^2 + c^2) (Eq. 2)."""
    s = np.asarray(s)
    xi, yi = np.asarray(centers[0], float), np.asarray(centers[1], float)
    Y, X = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    d = np.sqrt((X[None] - xi[:, None, None]) ** 2 + (Y[None] - yi[:, None, None]) ** 2 + c * c)
    return s[:, None, None] - d


def shift(g, design):
    """dphi = |smallest cone value on the design region| (g as from cones())."""
    return shift_of(g[:, np.asarray(design).astype(bool)])


def shift_of(g_design):
    return abs(np.min(np.real(g_design)))


def pnorm_levelset(s, centers, c, p, design, normalize=True, frozen=None):
    """(Phi (ny, nx), dphi, scale).  On the design region Phi = scale *
    ([sum_i (g_i + dphi)^p]^(1/p) - dphi); elsewhere Phi = 0 (the material
    there is fixed, so the level set is not used).  scale = 1 / max |.| over the
    design region, or 1 without renormalisation.  frozen = (dphi, scale)
    evaluates the map with both held at the given values (complex-step
    differentiation)."""
    D = np.asarray(design).astype(bool)
    ny, nx = D.shape
    g = cones(s, centers, c, nx, ny)[:, D]
    dphi = shift_of(g) if frozen is None else frozen[0]
    base = g + dphi
    vals = np.sum(base ** p, axis=0) ** (1.0 / p) - dphi
    if frozen is not None:
        scale = frozen[1]
    else:
        scale = 1.0 / np.max(np.abs(np.real(vals))) if normalize else 1.0
    phi = np.zeros((ny, nx), dtype=vals.dtype)
    phi[D] = scale * vals
    return phi, dphi, scale


def pnorm_levelset_vjp(s, centers, c, p, design, dJdphi, dphi, scale):
    """dJ/ds_i = scale * sum over design nodes of dJ/dPhi * ((g_i + dphi) / S)^(p - 1),
    S the p-norm [sum_j (g_j + dphi)^p]^(1/p); dphi and scale held fixed."""
    D = np.asarray(design).astype(bool)
    ny, nx = D.shape
    base = cones(s, centers, c, nx, ny)[:, D] + dphi
    S = np.sum(base ** p, axis=0) ** (1.0 / p)
    # where every base is 0 the p-norm has its kink at the origin: such a node
    # contributes nothing (the zero subgradient)
    live = np.real(S) > 0
    w = (base[:, live] / S[None, live]) ** (p - 1)
    return scale * np.sum(w * np.asarray(dJdphi)[D][live][None], axis=1)


def adam_step(s, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1): returns (s, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return s - lr * mhat / (np.sqrt(vhat) + eps), m, v
