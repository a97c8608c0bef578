"""Forward map: effective field, LLG right-hand side, classic RK4, energies.

Oracle (test infrastructure only).  Plain float64 NumPy; every function also
accepts complex arrays (complex-step differentiation in the tests).

Discretisation (paper: Methods, "nodal finite-difference discretization").
Magnetisation lives on the nodes of an nx*ny*nz grid with spacings dx, dy, dz;
each node carries a control volume V = dx*dy*dz.  Material maps from the level
set (Eq. 4 and the paragraph after it): Ms_i = Ms*psi_i, A_i = A*psi_i,
K_i = K*psi_i.  The energy of the discrete state is

  E_ex = V * sum_edges A * (2 psi_i psi_j / (psi_i + psi_j)) |m_j - m_i|^2 / h^2
  E_d  = 1/2 mu0 V sum_i Ms_i m_i . sum_j N(r_i - r_j) Ms_j m_j
  E_Z  = -V sum_i Ms_i m_i . B_ext,i(t)
  E_an = -V sum_i K_i (m_i . u)^2

and the effective field is B_i = -(1/(Ms_i V)) dE/dm_i (tesla).  Time
evolution is the LLG equation (Eq. 11) in its explicit Landau-Lifshitz form
dm/dt = -gamma' [m x B + alpha m x (m x B)], gamma' = gamma/(1+alpha^2), which
equals Eq. 11 for |m| = 1; nodes with psi = 0 are frozen (optionally every
node with psi <= psi_freeze, a threshold beyond the paper that removes the
dynamics of nearly massless interface nodes).  Time stepping is the classic
fourth-order Runge-Kutta method with a fixed step.
"""
from __future__ import annotations

import math

import numpy as np

from . import newell

MU0 = 4e-7 * math.pi

TERM_EXCH, TERM_DEMAG, TERM_ZEEMAN, TERM_ANIS = 1, 2, 4, 8


def _padded(n):
    """Smallest power of two >= 2n - 1 (1 for a single node)."""
    if n == 1:
        return 1
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p


class DemagKernel:
    """Zero-padded FFT form of the linear convolution x -> N * x on the grid."""

    def __init__(self, nx, ny, nz, h, pad=None):
        self.n = (nz, ny, nx)
        self.P = pad if pad is not None else (_padded(nz), _padded(ny), _padded(nx))
        Nq = newell.tensor_grid(nx, ny, nz, h)          # (6, nz, ny, nx) octant
        Pz, Py, Px = self.P
        K = np.zeros((6, Pz, Py, Px))
        for c in range(6):
            for sz in (1, -1):
                for sy in (1, -1):
                    for sx in (1, -1):
                        par = newell.PARITY[c]
                        sign = (par[0] if sx < 0 else 1) * (par[1] if sy < 0 else 1) * (par[2] if sz < 0 else 1)
                        iz = np.arange(nz) if sz > 0 else (-np.arange(nz)) % Pz
                        iy = np.arange(ny) if sy > 0 else (-np.arange(ny)) % Py
                        ix = np.arange(nx) if sx > 0 else (-np.arange(nx)) % Px
                        K[c][np.ix_(iz, iy, ix)] = sign * Nq[c]
        self.Khat = np.fft.rfftn(K, axes=(1, 2, 3))
        self.tensor_octant = Nq

    def _conv_real(self, x):
        nz, ny, nx = self.n
        Pz, Py, Px = self.P
        X = np.fft.rfftn(x, s=(Pz, Py, Px), axes=(1, 2, 3))
        xx, yy, zz, xy, xz, yz = self.Khat
        Y = np.stack([xx * X[0] + xy * X[1] + xz * X[2],
                      xy * X[0] + yy * X[1] + yz * X[2],
                      xz * X[0] + yz * X[1] + zz * X[2]])
        return np.fft.irfftn(Y, s=(Pz, Py, Px), axes=(1, 2, 3))[:, :nz, :ny, :nx]

    def conv(self, x):
        """(N * x)_i = sum_j N(r_i - r_j) x_j for a 3-vector field x (3, nz, ny, nx)."""
        if np.iscomplexobj(x):
            return self._conv_real(x.real) + 1j * self._conv_real(x.imag)
        return self._conv_real(x)


def demag_direct(x, h):
    """O(N^2) direct sum of sum_j N(r_i - r_j) x_j (tiny grids only)."""
    _, nz, ny, nx = x.shape
    out = np.zeros(x.shape, dtype=np.result_type(x, float))
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    xs = x.reshape(3, -1)
    for a in range(pos.shape[0]):
        d = pos[a] - pos
        Nt = newell.tensor_at(d[:, 0] * h[0], d[:, 1] * h[1], d[:, 2] * h[2], h)
        xx, yy, zz, xy, xz, yz = Nt
        o = out.reshape(3, -1)
        o[0, a] = (xx * xs[0] + xy * xs[1] + xz * xs[2]).sum()
        o[1, a] = (xy * xs[0] + yy * xs[1] + yz * xs[2]).sum()
        o[2, a] = (xz * xs[0] + yz * xs[1] + zz * xs[2]).sum()
    return out


def cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


class Sim:
    """One problem instance: parameters, masks and the demag kernel.

    ``prob`` is any object with the attributes of a workload Problem (nx, ny,
    nz, dx, dy, dz, Ms, A, K, ku, gamma, alpha0, alpha_max, ramp_cells,
    ramp_faces, B0, b_rf, f1, f2, t_switch, terms, dt)."""

    def __init__(self, prob, antenna=None, pad=None):
        self.p = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.h = (prob.dx, prob.dy, prob.dz)
        self.V = prob.dx * prob.dy * prob.dz
        self.terms = prob.terms
        self.kappa = 2.0 * prob.A / prob.Ms
        self.antenna = np.zeros(self.shape) if antenna is None else np.asarray(antenna, float)
        self.alpha = self._alpha_map()
        self.gp = prob.gamma / (1.0 + self.alpha ** 2)
        self.psi_freeze = float(getattr(prob, "psi_freeze", 0.0))
        self.demag = DemagKernel(prob.nx, prob.ny, prob.nz, self.h, pad) if prob.terms & TERM_DEMAG else None
        ku = np.asarray(prob.ku, float)
        self.u = ku / np.linalg.norm(ku) if np.linalg.norm(ku) > 0 else ku

    # -- material and source maps ------------------------------------------
    def _alpha_map(self):
        """Linear absorbing ramp: alpha0 + (alpha_max - alpha0) * max(0, (W - d)/W),
        d = node-index distance to the nearest ramped face."""
        p = self.p
        nz, ny, nx = self.shape
        W = p.ramp_cells
        alpha = np.full(self.shape, float(p.alpha0))
        if W <= 0 or p.ramp_faces == 0:
            return alpha
        kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        big = 10 ** 9
        d = np.full(self.shape, big)
        faces = [(1, ii), (2, nx - 1 - ii), (4, jj), (8, ny - 1 - jj), (16, kk), (32, nz - 1 - kk)]
        for bit, dist in faces:
            if p.ramp_faces & bit:
                d = np.minimum(d, dist)
        ramp = np.maximum(0.0, (W - d) / W)
        return p.alpha0 + (p.alpha_max - p.alpha0) * ramp

    def drive(self, t):
        """Scalar drive waveform.  sin(phase(t)), the frequency switching from f1
        to f2 at t_switch (if t_switch > 0) with a continuous phase; without a
        switch and with f2 > 0, the two-tone excitation of the demultiplexer
        section, sin(2 pi f1 t) + sin(2 pi f2 t).  drive_kind 1: the ramp t / t_ramp
        (with b_rf the field reached at t_ramp)."""
        p = self.p
        if getattr(p, "drive_kind", 0) == 1:
            # the linear field ramp of the magnetisation-curve experiment: 0 at t = 0, 1 at t_ramp
            return t / p.t_ramp
        if p.t_switch > 0 and t >= p.t_switch:
            ph = 2 * math.pi * (p.f1 * p.t_switch + p.f2 * (t - p.t_switch))
        elif p.t_switch <= 0 and p.f2 > 0:
            return math.sin(2 * math.pi * p.f1 * t) + math.sin(2 * math.pi * p.f2 * t)
        else:
            ph = 2 * math.pi * p.f1 * t
        return math.sin(ph)

    # -- field terms ------------------------------------------------------
    def _edges(self):
        """(axis, h, slice_a, slice_b) for every grid axis with more than one node."""
        nz, ny, nx = self.shape
        out = []
        for ax, n, h in ((3, nx, self.h[0]), (2, ny, self.h[1]), (1, nz, self.h[2])):
            if n > 1:
                a = [slice(None)] * 4
                b = [slice(None)] * 4
                a[ax] = slice(0, n - 1)
                b[ax] = slice(1, n)
                out.append((ax, h, tuple(a), tuple(b)))
        return out

    @staticmethod
    def _pair(psi, ax, h):
        """psi on both ends of every edge along ``ax`` and the edge sum."""
        sl_a = [slice(None)] * 3
        sl_b = [slice(None)] * 3
        n = psi.shape[ax - 1]
        sl_a[ax - 1] = slice(0, n - 1)
        sl_b[ax - 1] = slice(1, n)
        pa, pb = psi[tuple(sl_a)], psi[tuple(sl_b)]
        s = pa + pb
        nz = (s != 0)
        ssafe = np.where(nz, s, 1.0)
        return pa, pb, ssafe, nz

    def exchange_field(self, m, psi):
        """B_ex,i = kappa sum_j c_ij (m_j - m_i), c_ij = 2 psi_j / ((psi_i + psi_j) h^2)."""
        B = np.zeros(m.shape, dtype=np.result_type(m, psi, float))
        for ax, h, a, b in self._edges():
            pa, pb, s, nz = self._pair(psi, ax, h)
            dm = m[b] - m[a]
            cab = np.where(nz, 2.0 * pb / (s * h * h), 0.0)
            cba = np.where(nz, 2.0 * pa / (s * h * h), 0.0)
            B[a] += self.kappa * cab * dm
            B[b] -= self.kappa * cba * dm
        return B

    def demag_field(self, m, psi):
        """B_d = -mu0 Ms * N * (psi m)."""
        return -MU0 * self.p.Ms * self.demag.conv(psi * m)

    def zeeman_field(self, t):
        p = self.p
        B = np.zeros((3,) + self.shape)
        dv = self.drive(t)
        for c in range(3):
            B[c] = p.B0[c] + p.b_rf[c] * dv * self.antenna
        return B

    def anis_field(self, m):
        coef = 2.0 * self.p.K / self.p.Ms
        mu = dot(m, self.u[:, None, None, None])
        return coef * mu * self.u[:, None, None, None]

    def field(self, m, psi, t, terms=None):
        terms = self.terms if terms is None else terms
        B = np.zeros(m.shape, dtype=np.result_type(m, psi, float))
        if terms & TERM_EXCH:
            B = B + self.exchange_field(m, psi)
        if terms & TERM_DEMAG:
            B = B + self.demag_field(m, psi)
        if terms & TERM_ZEEMAN:
            B = B + self.zeeman_field(t)
        if terms & TERM_ANIS:
            B = B + self.anis_field(m)
        return B

    # -- dynamics ---------------------------------------------------------
    def frozen(self, psi):
        """Nodes without dynamics: psi = 0, or psi <= psi_freeze when that is set
        (compared on the real part, so complex steps do not move the set)."""
        if self.psi_freeze > 0:
            return np.real(psi) <= self.psi_freeze
        return psi == 0

    def rhs_from_field(self, m, B, psi):
        c = cross(m, B)
        f = -self.gp * (c + self.alpha * cross(m, c))
        return np.where(self.frozen(psi), 0.0, f)

    def rhs(self, m, psi, t):
        B = self.field(m, psi, t)
        return self.rhs_from_field(m, B, psi), B

    def rk4_step(self, m, psi, t):
        """One classic RK4 step; returns m_{n+1} and the stage states and fields."""
        dt = self.p.dt
        k1, B1 = self.rhs(m, psi, t)
        y2 = m + 0.5 * dt * k1
        k2, B2 = self.rhs(y2, psi, t + 0.5 * dt)
        y3 = m + 0.5 * dt * k2
        k3, B3 = self.rhs(y3, psi, t + 0.5 * dt)
        y4 = m + dt * k3
        k4, B4 = self.rhs(y4, psi, t + dt)
        m_next = m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return m_next, (m, y2, y3, y4), (B1, B2, B3, B4)

    def integrate(self, m0, psi, n_steps, t0=0.0, keep=False):
        """n_steps RK4 steps from m0 at time t0; t_n = t0 + n dt."""
        m = m0
        traj = [m0] if keep else None
        for n in range(n_steps):
            m, _, _ = self.rk4_step(m, psi, t0 + n * self.p.dt)
            if keep:
                traj.append(m)
        return (m, traj) if keep else m

    # -- energies ---------------------------------------------------------
    def energies(self, m, psi, t, terms=None):
        """Energy terms (J) of the discrete state, from their definitions."""
        terms = self.terms if terms is None else terms
        p = self.p
        V = self.V
        e = dict(ex=0.0, d=0.0, Z=0.0, an=0.0)
        if terms & TERM_EXCH:
            tot = 0.0
            for ax, h, a, b in self._edges():
                pa, pb, s, nz = self._pair(psi, ax, h)
                dm = m[b] - m[a]
                hm = np.where(nz, 2.0 * pa * pb / s, 0.0)
                tot = tot + (hm * dot(dm, dm)).sum() / (h * h)
            e["ex"] = V * p.A * tot
        if terms & TERM_DEMAG:
            Mv = p.Ms * psi * m
            e["d"] = 0.5 * MU0 * V * (dot(Mv, self.demag.conv(Mv))).sum()
        if terms & TERM_ZEEMAN:
            e["Z"] = -V * p.Ms * (psi * dot(m, self.zeeman_field(t))).sum()
        if terms & TERM_ANIS:
            mu = dot(m, self.u[:, None, None, None])
            e["an"] = -V * p.K * (psi * mu * mu).sum()
        e["tot"] = e["ex"] + e["d"] + e["Z"] + e["an"]
        return e
