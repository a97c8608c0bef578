"""Seeded synthetic workloads for the level-set LLG inverse-design path.

This module only *generates inputs*: grid sizes, material constants, masks,
initial magnetisation and initial level-set functions.  It holds none of the
method's arithmetic (no fields, no time stepping, no gradients), so both the
HIP library (through its Python binding) and the CPU oracle can take their
inputs from here without sharing any computation.

Material constants follow the paper's workloads: permalloy-like particle
(Ms = 800 kA/m, A = 13 pJ/m; "Stoner-Wohlfarth particle" section) and YIG
(Ms = 140 kA/m, A = 3.5 pJ/m; "Demultiplexer example" section).  Geometry of
the demultiplexer stand-in (input guide, square design region, two output
guides, antenna and port windows) is a synthetic layout with the structure of
the paper's Fig. 5 device, scaled to the grid of each workload.

All random draws use NumPy's PCG64 generator with an explicit seed and are
returned as arrays, so the GPU path and the oracle consume identical inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# term bitmask (mirrors LLG_TERM_* in include/llg.h)
TERM_EXCH = 1
TERM_DEMAG = 2
TERM_ZEEMAN = 4
TERM_ANIS = 8
TERM_ALL = TERM_EXCH | TERM_DEMAG | TERM_ZEEMAN | TERM_ANIS

# damping-ramp face bitmask (mirrors LLG_FACE_*)
FACE_XLO, FACE_XHI, FACE_YLO, FACE_YHI, FACE_ZLO, FACE_ZHI = 1, 2, 4, 8, 16, 32

OBJ_NONE = 0
OBJ_ENERGY_AREA = 1
OBJ_PORT_MY2 = 2
OBJ_PORT_SPECTRAL = 3
OBJ_MAG_CURVE = 4


@dataclasses.dataclass
class Problem:
    """Physical and numerical parameters of one LLG instance (SI units)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    Ms: float                   # saturation magnetisation of the full material, A/m
    A: float                    # exchange stiffness, J/m
    K: float = 0.0              # uniaxial anisotropy constant, J/m^3
    ku: tuple = (1.0, 0.0, 0.0)  # anisotropy axis (unit vector)
    gamma: float = 1.76e11      # gyromagnetic ratio, rad/(s T)
    alpha0: float = 1e-3        # Gilbert damping in the bulk
    alpha_max: float = 1e-3     # damping at a ramped face
    ramp_cells: int = 0         # width of the absorbing ramp, in nodes
    ramp_faces: int = 0         # FACE_* bitmask
    B0: tuple = (0.0, 0.0, 0.0)  # uniform bias field, T
    b_rf: tuple = (0.0, 0.0, 0.0)  # drive amplitude on the antenna mask, T
    f1: float = 0.0             # drive frequency before t_switch, Hz
    f2: float = 0.0             # drive frequency after t_switch, Hz
    t_switch: float = -1.0      # < 0: no switch
    terms: int = TERM_ALL
    dt: float = 1e-13
    drive_kind: int = 0         # 0: sine (switch / two tones as above); 1: linear ramp t / t_ramp
    t_ramp: float = 0.0         # duration of the ramp (drive_kind 1), s
    psi_freeze: float = 0.0     # nodes with psi <= psi_freeze carry no dynamics (0: psi = 0 only)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


@dataclasses.dataclass
class Workload:
    """A problem plus its seeded inputs and run settings."""
    name: str
    problem: Problem
    n_steps: int
    dtype: str                 # "f32" or "f64": precision of the GPU run
    heaviside_a: float         # slope a of the smoothed Heaviside psi = 1/(1+exp(-a*phi))
    phi: np.ndarray            # level-set function, shape (ny, nx) if extruded else (nz, ny, nx)
    extrude_z: bool
    design: np.ndarray         # u8 (nz, ny, nx): 1 where psi follows the level set
    psi_fixed: np.ndarray      # (nz, ny, nx): psi outside the design region
    antenna: np.ndarray        # u8 (nz, ny, nx)
    port1: np.ndarray          # u8 (nz, ny, nx)
    port2: np.ndarray          # u8 (nz, ny, nx)
    m0: np.ndarray             # (3, nz, ny, nx), unit vectors
    objective: int = OBJ_NONE
    obj_lambda: float = 1.0
    obj_area: float = 0.4
    obj_n_start: int = 0
    fd_nodes: Optional[np.ndarray] = None   # flat indices into phi for FD checks
    extra: Dict = dataclasses.field(default_factory=dict)


MU0_NOMINAL = 4e-7 * math.pi  # only used to state E_ref in workload metadata


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / np.sqrt((v * v).sum(axis=0, keepdims=True))


def _gaussian_filter2d(a: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur with reflecting borders (input generation only)."""
    r = int(math.ceil(4 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    k /= k.sum()
    out = a
    for axis in (0, 1):
        pad = [(0, 0), (0, 0)]
        pad[axis] = (r, r)
        p = np.pad(out, pad, mode="symmetric")
        acc = np.zeros_like(out)
        for i, w in enumerate(k):
            sl = [slice(None), slice(None)]
            sl[axis] = slice(i, i + out.shape[axis])
            acc += w * p[tuple(sl)]
        out = acc
    return out


def demux_layout(nx: int, ny: int, nz: int, D: int, wg: int, W: int):
    """Masks of the demultiplexer stand-in.

    Input guide on the left, a D x D design square in the middle, two output
    guides (port 1 at the top edge of the square, port 2 at the bottom edge) on
    the right; antenna a 3-node strip of the input guide just inside the
    absorbing ramp; port windows a 5-node strip of each output guide just
    before the right ramp.  Air (psi_fixed = 0) elsewhere.
    """
    yc = ny // 2
    xd0 = (nx - D) // 2
    y0, y1 = yc - D // 2, yc - D // 2 + D
    gi0 = yc - wg // 2
    shape2 = (ny, nx)
    guide = np.zeros(shape2, np.uint8)
    design = np.zeros(shape2, np.uint8)
    ant = np.zeros(shape2, np.uint8)
    p1 = np.zeros(shape2, np.uint8)
    p2 = np.zeros(shape2, np.uint8)
    guide[gi0:gi0 + wg, 0:xd0] = 1
    design[y0:y1, xd0:xd0 + D] = 1
    guide[y1 - wg:y1, xd0 + D:] = 1
    guide[y0:y0 + wg, xd0 + D:] = 1
    ant[gi0:gi0 + wg, W + 2:W + 5] = 1
    px0, px1 = nx - W - 8, nx - W - 3
    p1[y1 - wg:y1, px0:px1] = 1
    p2[y0:y0 + wg, px0:px1] = 1
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    return dict(design=rep(design), psi_fixed=rep(guide.astype(np.float64)),
                antenna=rep(ant), port1=rep(p1), port2=rep(p2),
                design2d=design, box=(xd0, y0, D))


def random_design_phi(rng: np.random.Generator, ny: int, nx: int, box, sigma: float = 4.0):
    """Smooth random level-set on the design square, max |phi| = 1, zero elsewhere."""
    xd0, y0, D = box
    xi = rng.standard_normal((D, D))
    s = _gaussian_filter2d(xi, sigma)
    s /= np.abs(s).max()
    phi = np.zeros((ny, nx))
    phi[y0:y0 + D, xd0:xd0 + D] = s
    return phi


def rbf_layout(box, n_side: int = 20, holes: int = 4, seed: int = 0, p: float = 90.0):
    """RBF parameterisation of a square design region box = (x0, y0, D) (nodes):
    n_side x n_side centres evenly spaced over it (the paper's 20 x 20 array),
    shape constant c = centre spacing h, and initial amplitudes forming a
    holes x holes grid of holes (the paper's 4 x 4 initial design): s = 1.5 h
    (material everywhere: the worst point between four centres still has a
    positive cone) except -1.5 h for centres within 2 h of a hole centre, plus a
    seeded U(-0.05, 0.05) h jitter.  holes = 0 gives a jittered uniform start."""
    x0, y0, D = box
    h = D / n_side
    k = (np.arange(n_side) + 0.5) * h
    XC, YC = np.meshgrid(x0 - 0.5 + k, y0 - 0.5 + k, indexing="xy")
    xc, yc = XC.reshape(-1), YC.reshape(-1)
    s = np.full(xc.size, 1.5 * h)
    if holes > 0:
        hc = (np.arange(holes) + 0.5) * D / holes
        for hy in hc:
            for hx in hc:
                near = np.hypot(xc - (x0 - 0.5 + hx), yc - (y0 - 0.5 + hy)) <= 2.0 * h
                s[near] = -1.5 * h
    rng = np.random.default_rng(seed)
    s += rng.uniform(-0.05, 0.05, s.size) * h
    return dict(xc=xc, yc=yc, c=h, p=p, s=s)


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def yig_waveguide_plain(seed: int = 0, n_steps: int = 500) -> Workload:
    """64x16x1 nodes, 5x5x10 nm^3 cells, YIG, exchange + demag + 0.2 T bias
    along x; m0 along x with a seeded N(0, 1e-3) transverse perturbation.
    Plain forward integration in FP64 (500 RK4 steps, dt = 1e-13 s)."""
    rng = np.random.default_rng(seed)
    p = Problem(nx=64, ny=16, nz=1, dx=5e-9, dy=5e-9, dz=10e-9, Ms=1.4e5, A=3.5e-12,
                alpha0=1e-3, alpha_max=1e-3, B0=(0.2, 0.0, 0.0),
                terms=TERM_EXCH | TERM_DEMAG | TERM_ZEEMAN, dt=1e-13)
    sh = p.shape
    m0 = np.zeros((3,) + sh)
    m0[0] = 1.0
    m0[1] = rng.normal(0.0, 1e-3, sh)
    m0[2] = rng.normal(0.0, 1e-3, sh)
    m0 = _normalise(m0)
    ones = np.ones(sh)
    zeros8 = np.zeros(sh, np.uint8)
    return Workload(name="yig_waveguide_64x16_fp64", problem=p, n_steps=n_steps, dtype="f64",
                    heaviside_a=50.0, phi=np.zeros(sh), extrude_z=False, design=zeros8,
                    psi_fixed=ones, antenna=zeros8, port1=zeros8, port2=zeros8, m0=m0)


def yig_film_probe(seed: int = 5, nx: int = 1024, ny: int = 1024, n_steps: int = 20) -> Workload:
    """HBM-scale probe of the fused step: a 1024x1024x1 YIG film (5x5x10 nm^3
    cells), the waveguide physics (exchange + demag + 0.2 T bias along x), m0
    along x with a seeded N(0, 1e-3) transverse perturbation, FP32."""
    rng = np.random.default_rng(seed)
    p = Problem(nx=nx, ny=ny, nz=1, dx=5e-9, dy=5e-9, dz=10e-9, Ms=1.4e5, A=3.5e-12,
                alpha0=1e-3, alpha_max=1e-3, B0=(0.2, 0.0, 0.0),
                terms=TERM_EXCH | TERM_DEMAG | TERM_ZEEMAN, dt=1e-13)
    sh = p.shape
    m0 = np.zeros((3,) + sh)
    m0[0] = 1.0
    m0[1] = rng.normal(0.0, 1e-3, sh)
    m0[2] = rng.normal(0.0, 1e-3, sh)
    m0 = _normalise(m0)
    zeros8 = np.zeros(sh, np.uint8)
    return Workload(name=f"yig_film_probe_{nx}x{ny}", problem=p, n_steps=n_steps, dtype="f32",
                    heaviside_a=50.0, phi=np.zeros(sh), extrude_z=False, design=zeros8,
                    psi_fixed=np.ones(sh), antenna=zeros8, port1=zeros8, port2=zeros8, m0=m0)


def permalloy_particle(seed: int = 1, n_steps: int = 2000, nx: int = 64, ny: int = 64) -> Workload:
    """64x64x1 nodes, 2 nm cubes, permalloy-like (Ms = 8e5 A/m, A = 1.3e-11 J/m,
    alpha = 0.5), no applied field.  phi = seeded sum of 4 Gaussians (sigma = 8
    cells, amplitudes U(-1,1)); smoothed Heaviside of width eps = 1.5 cells
    (a = 2/eps).  Objective: final exchange + demag energy / E_ref plus
    lambda*(mean(psi) - 0.4)^2.  2000 RK4 steps, dt = 5e-14 s."""
    rng = np.random.default_rng(seed)
    p = Problem(nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=8e5, A=1.3e-11,
                alpha0=0.5, alpha_max=0.5, terms=TERM_EXCH | TERM_DEMAG, dt=5e-14)
    sh = p.shape
    amp = rng.uniform(-1.0, 1.0, 4)
    cen = rng.uniform(0.0, 1.0, (4, 2)) * np.array([nx, ny])
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phi2 = np.zeros((ny, nx))
    for k in range(4):
        phi2 += amp[k] * np.exp(-((xx - cen[k, 0]) ** 2 + (yy - cen[k, 1]) ** 2) / (2 * 8.0 ** 2))
    ang = math.radians(30.0)
    m0 = np.zeros((3,) + sh)
    m0[0] = math.cos(ang)
    m0[1] = math.sin(ang)
    m0 += rng.normal(0.0, 1e-3, m0.shape)
    m0 = _normalise(m0)
    fd_nodes = rng.choice(nx * ny, size=16, replace=False)
    ones8 = np.ones(sh, np.uint8)
    zeros8 = np.zeros(sh, np.uint8)
    eps = 1.5
    return Workload(name="permalloy_particle_64x64_grad", problem=p, n_steps=n_steps, dtype="f32",
                    heaviside_a=2.0 / eps, phi=phi2, extrude_z=True, design=ones8,
                    psi_fixed=np.zeros(sh), antenna=zeros8, port1=zeros8, port2=zeros8, m0=m0,
                    objective=OBJ_ENERGY_AREA, obj_lambda=1.0, obj_area=0.4, fd_nodes=fd_nodes)


def _yig_demux_problem(nx, ny, nz, dx, dy, dz, dt, f1, f2=0.0, t_switch=-1.0, W=20):
    return Problem(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, Ms=1.4e5, A=3.5e-12,
                   alpha0=1e-3, alpha_max=0.5, ramp_cells=W, ramp_faces=FACE_XLO | FACE_XHI,
                   B0=(0.0, 0.0, 0.2), b_rf=(0.0, 1e-3, 0.0), f1=f1, f2=f2, t_switch=t_switch,
                   terms=TERM_EXCH | TERM_DEMAG | TERM_ZEEMAN, dt=dt)


def yig_demux(seed: int = 2, n_steps: int = 20000, nx: int = 256, ny: int = 96, f: float = 3e9,
              D: Optional[int] = None, wg: int = 20, dtype: str = "f32") -> Workload:
    """Demultiplexer stand-in: 256x96x1 nodes, 5x5x10 nm^3, YIG, 0.2 T bias
    perpendicular to the film, 1 mT sinusoidal drive at 3 GHz on the input
    antenna, absorbing damping ramp (1e-3 -> 0.5 over 20 nodes at the x faces),
    random-seeded phi on a 60x60-node (300x300 nm) design square.
    J = time average over the second half of the run of mean_{port1} m_y^2 -
    mean_{port2} m_y^2.  20 000 RK4 steps, dt = 1e-13 s."""
    rng = np.random.default_rng(seed)
    if D is None:
        D = min(60, ny - 4)
    p = _yig_demux_problem(nx, ny, 1, 5e-9, 5e-9, 10e-9, 1e-13, f)
    lay = demux_layout(nx, ny, 1, D, wg, p.ramp_cells)
    phi = random_design_phi(rng, ny, nx, lay["box"])
    m0 = np.zeros((3,) + p.shape)
    m0[2] = 1.0
    return Workload(name=f"yig_demux_{nx}x{ny}_grad", problem=p, n_steps=n_steps, dtype=dtype,
                    heaviside_a=50.0, phi=phi, extrude_z=True, design=lay["design"],
                    psi_fixed=lay["psi_fixed"], antenna=lay["antenna"], port1=lay["port1"],
                    port2=lay["port2"], m0=m0, objective=OBJ_PORT_MY2, obj_n_start=n_steps // 2,
                    extra=dict(box=lay["box"]))


def demux_windows(f1: float, f2: float, half_width: float, n_per_window: int):
    """Sample frequencies and weights of Eq. 10: n_per_window frequencies evenly
    spread over [f - half_width, f + half_width] around f1 and around f2.  Port 1
    is the top output (TO), port 2 the bottom one (BO), and
    J = (A_TO(f1) - A_BO(f1)) + (A_BO(f2) - A_TO(f2)): coef[0] weighs |X_TO|,
    coef[1] weighs |X_BO|."""
    w = np.linspace(-half_width, half_width, n_per_window) if n_per_window > 1 else np.zeros(1)
    freqs = np.concatenate([f1 + w, f2 + w])
    one = np.ones(n_per_window)
    coef = np.stack([np.concatenate([one, -one]), np.concatenate([-one, one])])
    return freqs, coef


def yig_demux_two_tone(seed: int = 2, n_steps: int = 20000, f1: float = 2.5e9, f2: float = 3.5e9,
                       half_width: float = 0.2e9, n_per_window: int = 5, dtype: str = "f32") -> Workload:
    """The demultiplexer driven by both tones at once (sin 2 pi f1 t + sin 2 pi
    f2 t on the antenna) with the spectral objective of Eq. 10 over the second
    half of the run: windows of n_per_window sample frequencies within
    +-half_width of f1 and f2.  2.5 / 3.5 GHz rather than the paper's 2.6 / 2.8
    GHz: the 1 ns window of a 20 000-step run resolves 1 GHz."""
    w = yig_demux(seed=seed, n_steps=n_steps, f=f1, dtype=dtype)
    w.problem.f2 = f2
    w.objective = OBJ_PORT_SPECTRAL
    freqs, coef = demux_windows(f1, f2, half_width, n_per_window)
    w.extra = dict(w.extra, freqs=freqs, coef=coef)
    w.name = f"yig_demux_{w.problem.nx}x{w.problem.ny}_spectral_grad"
    return w


def sw_particle_curve(seed: int = 6, n_steps: int = 2000, nx: int = 30, ny: int = 30) -> Workload:
    """The magnetisation-curve task (Eq. 8): 30x30x1 nodes of 3 nm, permalloy
    (Ms = 800 kA/m, A = 13 pJ/m), alpha = 0.5, the applied field ramped linearly
    along x from 0 to 0.3 Ms over the run; phi is seeded smooth noise (max |phi| = 1),
    and extra["rbf"] the 20x20 RBF array over the mesh with 3x3 holes for the
    design loop.  Target: the Stoner-Wohlfarth section's M = 2 H_ext, which is
    0.6 n / N in units of Ms at step n of the N-step ramp; weights
    1 / (target N); window = steps 1..N (the n = 0 term, whose target is 0, is
    left out)."""
    rng = np.random.default_rng(seed)
    dt = 1e-13
    mu0 = 4e-7 * math.pi
    p = Problem(nx=nx, ny=ny, nz=1, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5, A=1.3e-11, alpha0=0.5, alpha_max=0.5,
                b_rf=(0.3 * mu0 * 8e5, 0.0, 0.0), drive_kind=1, t_ramp=n_steps * dt,
                terms=TERM_EXCH | TERM_DEMAG | TERM_ZEEMAN, dt=dt)
    sh = p.shape
    lay = rbf_layout((0, 0, min(nx, ny)), n_side=20, holes=3, seed=seed)
    m0 = np.zeros((3,) + sh)
    m0[1] = 1.0
    m0 += rng.normal(0.0, 1e-3, m0.shape)
    m0 = _normalise(m0)
    target = 2.0 * 0.3 * np.arange(1, n_steps + 1) / n_steps
    ones8 = np.ones(sh, np.uint8)
    zeros8 = np.zeros(sh, np.uint8)
    phi = random_design_phi(rng, ny, nx, (0, 0, min(nx, ny)))
    w = Workload(name=f"sw_particle_{nx}x{ny}_curve_grad", problem=p, n_steps=n_steps, dtype="f32",
                 heaviside_a=50.0, phi=phi, extrude_z=True, design=ones8, psi_fixed=np.zeros(sh),
                 antenna=ones8, port1=zeros8, port2=zeros8, m0=m0, objective=OBJ_MAG_CURVE, obj_n_start=0,
                 extra=dict(rbf=lay, target=target, weight=1.0 / (target * n_steps)))
    return w


def yig_demux_sweep(seed: int = 3, n_designs: int = 32, freqs=(2.5e9, 3.5e9), n_steps: int = 10000) -> List[Workload]:
    """Batched sweep: n_designs independently seeded phi, each on its own grid
    with nx ~ U{128..256}, ny ~ U{64..128}, times the listed drive
    frequencies (both frequencies of a design share its grid and phi)."""
    rng = np.random.default_rng(seed)
    out = []
    for d in range(n_designs):
        nx = int(rng.integers(128, 257))
        ny = int(rng.integers(64, 129))
        dseed = int(rng.integers(0, 2 ** 31))
        for f in freqs:
            w = yig_demux(seed=dseed, n_steps=n_steps, nx=nx, ny=ny, f=f)
            w.name = f"sweep_d{d}_f{f / 1e9:.1f}GHz_{nx}x{ny}"
            out.append(w)
    return out


def yig_device_3d(seed: int = 4, n_steps: int = 50000, dtype: str = "f32",
                  nx: int = 512, ny: int = 256, nz: int = 4, D: int = 250, wg: int = 75) -> Workload:
    """Large 3D device: 512x256x4 nodes, 4x4x5 nm^3, YIG, full 3D demag, seeded
    random phi extruded through the thickness, drive at 2.5 GHz for the first
    half of the run then 3.5 GHz (phase-continuous).  dt = 8e-14 s."""
    rng = np.random.default_rng(seed)
    dt = 8e-14
    p = _yig_demux_problem(nx, ny, nz, 4e-9, 4e-9, 5e-9, dt, 2.5e9, 3.5e9, t_switch=(n_steps // 2) * dt)
    lay = demux_layout(nx, ny, nz, D, wg, p.ramp_cells)
    phi = random_design_phi(rng, ny, nx, lay["box"])
    m0 = np.zeros((3,) + p.shape)
    m0[2] = 1.0
    return Workload(name=f"yig_device3d_{nx}x{ny}x{nz}", problem=p, n_steps=n_steps, dtype=dtype,
                    heaviside_a=50.0, phi=phi, extrude_z=True, design=lay["design"],
                    psi_fixed=lay["psi_fixed"], antenna=lay["antenna"], port1=lay["port1"],
                    port2=lay["port2"], m0=m0, objective=OBJ_PORT_MY2, obj_n_start=n_steps // 2)


def energy_reference(w: Workload) -> float:
    """Normalisation energy 1/2 mu0 Ms^2 N V of the energy objective (a constant
    of the workload definition, stated here so both sides take the same value)."""
    p = w.problem
    return 0.5 * MU0_NOMINAL * p.Ms ** 2 * p.n * p.dx * p.dy * p.dz
