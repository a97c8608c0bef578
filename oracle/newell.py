"""Cell-averaged demagnetisation tensor of a regular grid of rectangular cells.

Oracle (test infrastructure only).

Definition.  For two cells of size dx x dy x dz whose centres are offset by
r = (X, Y, Z), the tensor N(r) relates the mean field in one cell to the
uniform magnetisation of the other: <H> = -N(r) M.  Written as an integral it
is N(r) = (1/V) * int T(s) D(r + s) ds, where V = dx dy dz,
T(s) = prod_d (h_d - |s_d|)_+ is the autocorrelation of the box (its integral
is V^2), and D(p) = -(3 p p^T / |p|^2 - I) / (4 pi |p|^3) is the point-dipole
kernel.  The paper's effective field contains this dipole-dipole term (Methods,
"effective field ... demagnetizing (dipole-dipole) field"); the tensor form is
the standard finite-difference discretisation of it.

Near field (cells closer than two cell sizes): Newell, Williams & Dunlop
(J. Geophys. Res. 98, 9551, 1993) closed form, a 27-point second difference of
the functions f (diagonal) and g (off-diagonal).  Far field: Gauss-Legendre
quadrature of the tent-weighted dipole integral above, split at s_d = 0 where
the tent has its kink.  The closed form loses ~eps*R^6 to cancellation, the
quadrature converges geometrically with distance, so the switch keeps the
whole tensor near double-precision rounding.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


# -- Newell closed form -------------------------------------------------------

def _asinh_ratio(num, den2):
    """asinh(num / sqrt(den2)) with den2 >= 0; returns 0 where den2 == 0."""
    den = np.sqrt(den2)
    safe = np.where(den2 > 0, den, 1.0)
    return np.where(den2 > 0, np.arcsinh(num / safe), 0.0)


def _atan_ratio(num, den):
    safe = np.where(den != 0, den, 1.0)
    return np.where(den != 0, np.arctan(num / safe), 0.0)


def newell_f(x, y, z):
    """Newell's f(x, y, z); its 27-point second difference gives N_xx."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    out = out + 0.5 * y * (z2 - x2) * _asinh_ratio(y, x2 + z2)
    out = out + 0.5 * z * (y2 - x2) * _asinh_ratio(z, x2 + y2)
    out = out - x * y * z * _atan_ratio(y * z, x * R)
    return out


def newell_g(x, y, z):
    """Newell's g(x, y, z); its 27-point second difference gives N_xy."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    out = out + x * y * z * _asinh_ratio(z, x2 + y2)
    out = out + y * (3.0 * z2 - y2) * _asinh_ratio(x, y2 + z2) / 6.0
    out = out + x * (3.0 * z2 - x2) * _asinh_ratio(y, x2 + z2) / 6.0
    out = out - z * z2 * _atan_ratio(x * y, z * R) / 6.0
    out = out - 0.5 * z * y2 * _atan_ratio(x * z, y * R)
    out = out - 0.5 * z * x2 * _atan_ratio(y * z, x * R)
    return out


def _second_difference(fun, X, Y, Z, hx, hy, hz):
    """sum over e in {-1,0,1}^3 of w(e) fun(X + ex hx, ...), w = prod (2 if 0 else -1)."""
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    w1 = {-1: -1.0, 0: 2.0, 1: -1.0}
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            for ez in (-1, 0, 1):
                w = w1[ex] * w1[ey] * w1[ez]
                acc = acc + w * fun(X + ex * hx, Y + ey * hy, Z + ez * hz)
    return acc


def newell_exact(X, Y, Z, h):
    """All six components (xx, yy, zz, xy, xz, yz) from the closed form."""
    hx, hy, hz = h
    c = 1.0 / (FOUR_PI * hx * hy * hz)
    nxx = c * _second_difference(newell_f, X, Y, Z, hx, hy, hz)
    nyy = c * _second_difference(newell_f, Y, X, Z, hy, hx, hz)
    nzz = c * _second_difference(newell_f, Z, Y, X, hz, hy, hx)
    nxy = c * _second_difference(newell_g, X, Y, Z, hx, hy, hz)
    nxz = c * _second_difference(newell_g, X, Z, Y, hx, hz, hy)
    nyz = c * _second_difference(newell_g, Y, Z, X, hy, hz, hx)
    return np.stack([nxx, nyy, nzz, nxy, nxz, nyz])


# -- far field: quadrature of the tent-weighted dipole kernel ----------------

def _tent_rule(h, n):
    """Nodes/weights on [-h, h] for int T(s) f(s) ds with T(s) = h - |s|,
    Gauss-Legendre with n points on each half."""
    t, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * h * (t + 1.0)           # nodes on [0, h]
    ws = 0.5 * h * w * (h - s)        # tent weight folded in
    return np.concatenate([-s[::-1], s]), np.concatenate([ws[::-1], ws])


def dipole_quadrature(X, Y, Z, h, n):
    """(1/V) int T(s) D(r + s) ds for arrays of offsets, n GL points per half-axis."""
    hx, hy, hz = h
    V = hx * hy * hz
    sx, wx = _tent_rule(hx, n)
    sy, wy = _tent_rule(hy, n)
    sz, wz = _tent_rule(hz, n)
    X = np.asarray(X, float)[..., None]
    Y = np.asarray(Y, float)[..., None]
    Z = np.asarray(Z, float)[..., None]
    out = np.zeros((6,) + X.shape[:-1])
    for jx in range(sx.size):
        px = X + sx[jx]
        for jy in range(sy.size):
            py = Y + sy[jy]
            wxy = wx[jx] * wy[jy]
            pz = Z + sz[None, :]
            r2 = px * px + py * py + pz * pz
            inv_r = 1.0 / np.sqrt(r2)
            inv_r3 = inv_r / r2
            inv_r5 = inv_r3 / r2
            w = wxy * wz[None, :]
            # D = -(3 p p^T / r^5 - I / r^3) / (4 pi)
            out[0] += ((inv_r3 - 3.0 * px * px * inv_r5) * w).sum(-1)
            out[1] += ((inv_r3 - 3.0 * py * py * inv_r5) * w).sum(-1)
            out[2] += ((inv_r3 - 3.0 * pz * pz * inv_r5) * w).sum(-1)
            out[3] += ((-3.0 * px * py * inv_r5) * w).sum(-1)
            out[4] += ((-3.0 * px * pz * inv_r5) * w).sum(-1)
            out[5] += ((-3.0 * py * pz * inv_r5) * w).sum(-1)
    return out / (FOUR_PI * V)


def _gap_ratio(X, Y, Z, h):
    """Euclidean distance from the origin to the support of T(s) shifted by r
    (the nearest singularity of the integrand), in units of the largest edge."""
    hx, hy, hz = h
    gx = np.maximum(np.abs(X) - hx, 0.0)
    gy = np.maximum(np.abs(Y) - hy, 0.0)
    gz = np.maximum(np.abs(Z) - hz, 0.0)
    return np.sqrt(gx * gx + gy * gy + gz * gz) / max(hx, hy, hz)


NEAR_GAP = 1.5   # closed form below this gap ratio, quadrature above


def tensor_at(X, Y, Z, h):
    """N(r) (6 components) at arrays of physical offsets (X, Y, Z)."""
    X, Y, Z = np.broadcast_arrays(np.asarray(X, float), np.asarray(Y, float), np.asarray(Z, float))
    out = np.zeros((6,) + X.shape)
    q = _gap_ratio(X, Y, Z, h)
    near = q < NEAR_GAP
    if near.any():
        out[:, near] = newell_exact(X[near], Y[near], Z[near], h)
    npts = np.where(q <= 8.0, 8, np.where(q <= 30.0, 5, 4))
    for n in (8, 5, 4):
        sel = (~near) & (npts == n)
        if sel.any():
            out[:, sel] = dipole_quadrature(X[sel], Y[sel], Z[sel], h, n)
    return out


def tensor_grid(nx, ny, nz, h):
    """N at every node offset (i, j, k) with 0 <= i < nx etc. (non-negative octant).

    The other octants follow from the parities: diagonal components are even in
    every offset; xy is odd in X and Y; xz odd in X and Z; yz odd in Y and Z.
    Returns an array (6, nz, ny, nx)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return tensor_at(i * h[0], j * h[1], k * h[2], h)


# parity of (xx, yy, zz, xy, xz, yz) under X -> -X, Y -> -Y, Z -> -Z
PARITY = np.array([[1, 1, 1], [1, 1, 1], [1, 1, 1], [-1, -1, 1], [-1, 1, -1], [1, -1, -1]])
