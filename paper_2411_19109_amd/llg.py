"""Thin ctypes binding of the HIP library (include/llg.h).

Argument marshalling only: every step of the path runs in the library's
kernels.  PyTorch supplies device memory (tensors on ``cuda``) and the current
HIP stream.  The library must have been built (``python -m
paper_2411_19109_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllg.so")

LLG_OK, LLG_EINVAL, LLG_ESHAPE, LLG_ENOMEM, LLG_EHIP, LLG_ENONFINITE, LLG_ENOTSUP, LLG_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
LLG_F32, LLG_F64 = 0, 1
LLG_CKPT_SQRT, LLG_CKPT_ALL, LLG_CKPT_BINOMIAL = 0, 1, 2
LLG_OBJ_NONE, LLG_OBJ_ENERGY_AREA, LLG_OBJ_PORT_MY2, LLG_OBJ_PORT_SPECTRAL, LLG_OBJ_MAG_CURVE = 0, 1, 2, 3, 4
LLG_DRIVE_SINE, LLG_DRIVE_RAMP = 0, 1

EXPORTS = ["llg_last_error", "llg_version", "llg_create", "llg_destroy", "llg_levelset_to_Ms",
           "llg_levelset_to_Ms_vjp", "llg_field", "llg_forward", "llg_objective", "llg_adjoint",
           "llg_query_memory", "llg_query_recompute", "llg_set_graphs", "llg_launch_config",
           "llg_set_launch_config", "llg_autotune", "llg_fft_sizes", "llg_profile", "llg_profile_read", "llg_batch_create",
           "llg_batch_destroy", "llg_batch_size", "llg_batch_levelset_to_Ms", "llg_batch_levelset_to_Ms_vjp",
           "llg_batch_forward", "llg_batch_adjoint", "llg_rbf_work_len", "llg_rbf_levelset", "llg_rbf_levelset_vjp",
           "llg_adam_step", "llg_rbf_profile", "llg_rbf_profile_read", "llg_shape_penalty", "llg_forward_adaptive",
           "llg_adaptive_steps", "llg_adjoint_adaptive", "llg_adjoint_continuous",
           "llg_set_keep_stages", "llg_demag_tensor", "llg_shape_penalty_noalloc"]
RBF_KIND_NAMES = {0: "k_rbf_cones", 1: "k_rbf_pnorm", 2: "k_rbf_vjp"}
KIND_STAGE_FWD, KIND_COLUMN, KIND_STAGE_BWD = 0, 1, 2
# kernel classes of llg_profile_read; the column class runs k_col2d on single-layer
# grids and k_col_conv on thicker ones
KIND_NAMES = {KIND_STAGE_FWD: "k_stage_fwd", KIND_COLUMN: "k_col", KIND_STAGE_BWD: "k_stage_bwd"}


class LLGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"llg error {code}: {msg}")
        self.code = code


class Problem_c(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("Ms", ctypes.c_double), ("A", ctypes.c_double), ("K", ctypes.c_double),
                ("ku", ctypes.c_double * 3), ("gamma", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("ramp_cells", ctypes.c_int32), ("ramp_faces", ctypes.c_int32),
                ("B0", ctypes.c_double * 3), ("b_rf", ctypes.c_double * 3),
                ("f1", ctypes.c_double), ("f2", ctypes.c_double), ("t_switch", ctypes.c_double),
                ("terms", ctypes.c_int32), ("dtype", ctypes.c_int32), ("dt", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("ckpt_policy", ctypes.c_int32), ("ckpt_param", ctypes.c_int32),
                ("drive_kind", ctypes.c_int32), ("t_ramp", ctypes.c_double), ("psi_freeze", ctypes.c_double)]


class Masks_c(ctypes.Structure):
    _fields_ = [("antenna", ctypes.c_void_p), ("port1", ctypes.c_void_p), ("port2", ctypes.c_void_p),
                ("design", ctypes.c_void_p)]


class Objective_c(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("E_ref", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("area", ctypes.c_double), ("n_start", ctypes.c_int64), ("n_freq", ctypes.c_int32),
                ("freqs", ctypes.POINTER(ctypes.c_double)), ("coef", ctypes.POINTER(ctypes.c_double)),
                ("target", ctypes.POINTER(ctypes.c_double)), ("weight", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    """Load libllg.so once (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_2411_19109_amd.build`)")
    # PyTorch ships its own HIP runtime; load it first so that the library binds
    # to the same libamdhip64 instance (one runtime per process).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.llg_last_error.restype = ctypes.c_char_p
    L.llg_version.restype = ctypes.c_char_p
    sig = {
        "llg_create": [ctypes.POINTER(Problem_c), ctypes.POINTER(Masks_c), ctypes.POINTER(vp)],
        "llg_destroy": [vp],
        "llg_levelset_to_Ms": [vp, vp, vp, dbl, ctypes.c_int, vp, vp],
        "llg_levelset_to_Ms_vjp": [vp, vp, vp, dbl, ctypes.c_int, vp, vp],
        "llg_field": [vp, vp, vp, dbl, vp, vp, vp],
        "llg_forward": [vp, vp, vp, dbl, i64, ctypes.POINTER(Objective_c), vp, vp, vp],
        "llg_objective": [vp, ctypes.POINTER(Objective_c), vp, vp, dbl, vp, vp, vp, vp, vp],
        "llg_adjoint": [vp, vp, vp, vp, ctypes.POINTER(Objective_c), vp, vp, vp],
        "llg_query_memory": [ctypes.POINTER(Problem_c), i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "llg_query_recompute": [i64, i32, i32, ctypes.POINTER(i64)],
        "llg_fft_sizes": [vp, ctypes.POINTER(ctypes.c_int32)],
        "llg_profile": [vp, ctypes.c_int],
        "llg_set_graphs": [vp, ctypes.c_int],
        "llg_launch_config": [vp, ctypes.POINTER(i32)],
        "llg_set_launch_config": [vp, ctypes.POINTER(i32)],
        "llg_autotune": [vp, vp],
        "llg_batch_create": [ctypes.POINTER(Problem_c), ctypes.POINTER(Masks_c), i32, ctypes.POINTER(vp)],
        "llg_batch_destroy": [vp],
        "llg_batch_size": [vp, ctypes.POINTER(i32)],
        "llg_batch_levelset_to_Ms": [vp, vp, vp, dbl, ctypes.c_int, vp, vp],
        "llg_batch_levelset_to_Ms_vjp": [vp, vp, vp, dbl, ctypes.c_int, vp, vp],
        "llg_batch_forward": [vp, vp, vp, dbl, i64, ctypes.POINTER(Objective_c), vp, vp, vp],
        "llg_batch_adjoint": [vp, vp, vp, vp, ctypes.POINTER(Objective_c), vp, vp, vp],
        "llg_profile_read": [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.c_int],
        "llg_rbf_work_len": [i32, i32, i32, ctypes.POINTER(i64)],
        "llg_rbf_levelset": [i32, i32, i32, i32, vp, vp, dbl, dbl, vp, ctypes.c_int, vp, vp, vp, vp],
        "llg_rbf_levelset_vjp": [i32, i32, i32, i32, vp, vp, dbl, dbl, vp, vp, vp, vp, vp, vp],
        "llg_adam_step": [i32, vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, vp],
        "llg_rbf_profile": [ctypes.c_int],
        "llg_shape_penalty": [vp, vp, dbl, dbl, dbl, dbl, dbl, vp, vp, vp],
        "llg_shape_penalty_noalloc": [vp, vp, dbl, dbl, dbl, dbl, dbl, vp, vp, vp],
        "llg_forward_adaptive": [vp, vp, vp, dbl, dbl, dbl, dbl, dbl, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp],
        "llg_adaptive_steps": [vp, ctypes.POINTER(dbl), i64],
        "llg_adjoint_adaptive": [vp, vp, vp, vp, vp, vp, vp],
        "llg_adjoint_continuous": [vp, vp, vp, vp, ctypes.c_int, vp, vp, vp],
        "llg_set_keep_stages": [vp, ctypes.c_int],
        "llg_demag_tensor": [dbl, dbl, dbl, dbl, dbl, dbl, i32, ctypes.POINTER(dbl)],
        "llg_rbf_profile_read": [i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.c_int],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = L
    return L


def check(rc):
    if rc != LLG_OK:
        raise LLGError(rc, lib().llg_last_error().decode())


def make_problem(prob, dtype="f32", max_steps=1, ckpt_policy=LLG_CKPT_SQRT, ckpt_param=0) -> Problem_c:
    """Problem_c from any object with the attributes of workloads.Problem."""
    c = Problem_c()
    c.nx, c.ny, c.nz = prob.nx, prob.ny, prob.nz
    c.dx, c.dy, c.dz = prob.dx, prob.dy, prob.dz
    c.Ms, c.A, c.K = prob.Ms, prob.A, prob.K
    c.ku = (ctypes.c_double * 3)(*prob.ku)
    c.gamma = prob.gamma
    c.alpha0, c.alpha_max = prob.alpha0, prob.alpha_max
    c.ramp_cells, c.ramp_faces = prob.ramp_cells, prob.ramp_faces
    c.B0 = (ctypes.c_double * 3)(*prob.B0)
    c.b_rf = (ctypes.c_double * 3)(*prob.b_rf)
    c.f1, c.f2, c.t_switch = prob.f1, prob.f2, prob.t_switch
    c.terms = prob.terms
    c.dtype = LLG_F64 if dtype in ("f64", "float64", LLG_F64) else LLG_F32
    c.dt = prob.dt
    c.max_steps = max_steps
    c.ckpt_policy = ckpt_policy
    c.ckpt_param = ckpt_param
    c.drive_kind = getattr(prob, "drive_kind", LLG_DRIVE_SINE)
    c.t_ramp = getattr(prob, "t_ramp", 0.0)
    c.psi_freeze = getattr(prob, "psi_freeze", 0.0)
    return c


def make_objective(kind=LLG_OBJ_NONE, E_ref=1.0, lam=1.0, area=0.4, n_start=0, freqs=None, coef=None, target=None,
                   weight=None) -> Objective_c:
    """Objective_c; for LLG_OBJ_PORT_SPECTRAL, freqs (K sample frequencies, Hz)
    and coef (2 x K weights of |X_1(f_q)| and |X_2(f_q)|); for LLG_OBJ_MAG_CURVE,
    target and weight (one value per window step).  The object keeps its arrays
    alive."""
    o = Objective_c()
    o.kind, o.E_ref, o.lambda_, o.area, o.n_start = kind, E_ref, lam, area, n_start
    keep = []
    if target is not None:
        tg = np.ascontiguousarray(np.asarray(target, np.float64).reshape(-1))
        wt = np.ascontiguousarray(np.asarray(weight, np.float64).reshape(-1))
        if wt.size != tg.size:
            raise ValueError("target and weight must have one value per window step")
        keep += [tg, wt]
        o.target = tg.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.weight = wt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    o._keep_curve = keep
    if freqs is not None:
        f = np.ascontiguousarray(np.asarray(freqs, np.float64).reshape(-1))
        c = np.ascontiguousarray(np.asarray(coef, np.float64).reshape(-1))
        if c.size != 2 * f.size:
            raise ValueError("coef must hold 2 x len(freqs) weights")
        o._keep = (f, c)
        o.n_freq = f.size
        o.freqs = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.coef = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return o


def _check_obj(obj, n_steps):
    """The curve objective's host arrays are read for n_steps - n_start window
    steps: refuse shorter ones before the library reads them."""
    if obj is not None and obj.kind == LLG_OBJ_MAG_CURVE:
        keep = getattr(obj, "_keep_curve", [])
        if not keep or keep[0].size != n_steps - obj.n_start:
            raise ValueError("curve objective: target and weight need n_steps - n_start values")


def query_memory(prob, n_steps, policy=LLG_CKPT_SQRT, ckpt_param=0, dtype="f32") -> int:
    b = ctypes.c_size_t(0)
    check(lib().llg_query_memory(ctypes.byref(make_problem(prob, dtype, max(1, n_steps))), n_steps, policy,
                                 ckpt_param, ctypes.byref(b)))
    return b.value


def query_recompute(n_steps, policy=LLG_CKPT_SQRT, ckpt_param=0) -> int:
    """Forward RK4 steps the adjoint recomputes after a forward run of n_steps."""
    v = ctypes.c_int64(0)
    check(lib().llg_query_recompute(n_steps, policy, ckpt_param, ctypes.byref(v)))
    return v.value


def demag_tensor(h, r, method=0):
    """The library's demagnetising tensor between cells of edges h = (dx, dy, dz)
    whose centres are r = (X, Y, Z) apart (host float64): N_xx, N_yy, N_zz,
    N_xy, N_xz, N_yz.  method 0 as the library builds it, 1 closed form,
    2 quadrature."""
    out = (ctypes.c_double * 6)()
    check(lib().llg_demag_tensor(float(h[0]), float(h[1]), float(h[2]), float(r[0]), float(r[1]), float(r[2]),
                                 int(method), out))
    return np.array(out[:], dtype=np.float64)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One problem instance on the current HIP device (wraps llg_handle)."""

    def __init__(self, prob, dtype="f32", max_steps=1, antenna=None, port1=None, port2=None, design=None,
                 ckpt_policy=LLG_CKPT_SQRT, ckpt_param=0):
        import torch
        self.prob = prob
        self.dtype = dtype
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        self.N = prob.nx * prob.ny * prob.nz
        self._pc = make_problem(prob, dtype, max_steps, ckpt_policy, ckpt_param)
        keep = []

        def mask(a):
            if a is None:
                return None
            arr = np.ascontiguousarray(np.asarray(a, dtype=np.uint8).reshape(-1))
            if arr.size != self.N:
                raise ValueError("mask size mismatch")
            keep.append(arr)
            return arr.ctypes.data

        self._mk = Masks_c(mask(antenna), mask(port1), mask(port2), mask(design))
        h = ctypes.c_void_p()
        check(lib().llg_create(ctypes.byref(self._pc), ctypes.byref(self._mk), ctypes.byref(h)))
        self.h = h
        self._fwd_gen = 0  # counts the forward records (forward, autotune) on this handle
        del keep

    def close(self):
        if getattr(self, "h", None):
            lib().llg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------
    def _t(self, x, n):
        import torch
        if x.dtype != self.tdtype or not x.is_cuda or not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"expected a contiguous cuda tensor of {n} {self.tdtype}")
        return x

    def profile(self, enable, stride=1):
        """Event-time every stride-th launch of each kernel class while enable."""
        check(lib().llg_profile(self.h, int(stride) if enable else 0))

    def set_graphs(self, enable: bool):
        """Capture forward / adjoint launch sequences in HIP graphs and replay them."""
        check(lib().llg_set_graphs(self.h, int(enable)))

    def launch_config(self):
        """(column tile, column threads, column radix, forward row threads, forward radix,
        backward row threads, backward radix, staged values per row in the backward kernel)."""
        c = (ctypes.c_int32 * 8)()
        check(lib().llg_launch_config(self.h, c))
        return tuple(c)

    def set_launch_config(self, *cfg):
        """Eight values in the order of launch_config()."""
        c = (ctypes.c_int32 * 8)(*cfg)
        check(lib().llg_set_launch_config(self.h, c))

    def autotune(self):
        """Time the valid launch configurations and keep the fastest (drops the forward record)."""
        import torch
        check(lib().llg_autotune(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        self._fwd_gen += 1
        return self.launch_config()

    def profile_read(self, kind, reset=True):
        """(device ms, launches, algorithmic bytes) summed over profiled launches of one kernel class."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        check(lib().llg_profile_read(self.h, kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b), int(reset)))
        return ms.value, n.value, b.value

    def fft_sizes(self):
        a = (ctypes.c_int32 * 3)()
        check(lib().llg_fft_sizes(self.h, a))
        return tuple(a)

    # -- entry points ------------------------------------------------------
    def levelset_to_psi(self, phi, a, psi_fixed=None, extrude_z=True, out=None):
        import torch
        npsi = self.prob.nx * self.prob.ny if extrude_z else self.N
        self._t(phi, npsi)
        if psi_fixed is not None:
            self._t(psi_fixed, self.N)
        out = torch.empty(self.N, dtype=self.tdtype, device=phi.device) if out is None else out
        check(lib().llg_levelset_to_Ms(self.h, _ptr(phi), _ptr(psi_fixed), float(a), int(extrude_z), _ptr(out), _stream()))
        return out

    def levelset_vjp(self, phi, dJdpsi, a, extrude_z=True):
        import torch
        out = torch.empty(phi.numel(), dtype=torch.float64, device=phi.device)
        check(lib().llg_levelset_to_Ms_vjp(self.h, _ptr(phi), _ptr(dJdpsi), float(a), int(extrude_z), _ptr(out), _stream()))
        return out

    def forward_adaptive(self, psi, m0, t_end, h0, rtol, atol, t0=0.0):
        """Adaptive Dormand-Prince run to t_end: (m(t_end), accepted step sizes
        (numpy), rejected trials)."""
        import torch
        self._t(psi, self.N)
        self._t(m0, 3 * self.N)
        m_out = torch.empty_like(m0)
        na, nr = ctypes.c_int64(0), ctypes.c_int64(0)
        self._fwd_gen += 1
        check(lib().llg_forward_adaptive(self.h, _ptr(psi), _ptr(m0), float(t0), float(t_end), float(h0), float(rtol),
                                         float(atol), _ptr(m_out), ctypes.byref(na), ctypes.byref(nr), _stream()))
        hs = np.zeros(max(1, na.value))
        check(lib().llg_adaptive_steps(self.h, hs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), hs.size))
        return m_out, hs[:na.value], nr.value

    def set_keep_stages(self, keep: bool):
        """Adaptive runs keep every accepted step's stages for the adjoint
        (more device memory, no recomputation, bitwise-equal results)."""
        check(lib().llg_set_keep_stages(self.h, int(keep)))

    def adjoint_adaptive(self, psi, dJdm_T=None, dJdpsi_expl=None, want_dm0=False, continuous=False, n_sub=1):
        """Adjoint of the last adaptive run: discrete (exact for the accepted
        steps) or, with continuous=True, the continuous adjoint equation
        integrated backwards with n_sub RK4 steps per interval."""
        import torch
        dJdpsi = torch.empty(self.N, dtype=torch.float64, device=psi.device)
        dm0 = torch.empty(3 * self.N, dtype=self.tdtype, device=psi.device) if want_dm0 else None
        if continuous:
            check(lib().llg_adjoint_continuous(self.h, _ptr(psi), _ptr(dJdm_T), _ptr(dJdpsi_expl), int(n_sub),
                                               _ptr(dJdpsi), _ptr(dm0), _stream()))
        else:
            check(lib().llg_adjoint_adaptive(self.h, _ptr(psi), _ptr(dJdm_T), _ptr(dJdpsi_expl), _ptr(dJdpsi),
                                             _ptr(dm0), _stream()))
        return (dJdpsi, dm0) if want_dm0 else dJdpsi

    def shape_penalty(self, psi, xi, S_target, nu, x0, y0, want_grad=True):
        """(J, dJ/dpsi) of the size and centre constraints of Eq. 9 (device
        tensors; the gradient goes to adjoint(..., dJdpsi_expl=...))."""
        import torch
        self._t(psi, self.N)
        J = torch.zeros(1, dtype=torch.float64, device=psi.device)
        g = torch.empty(self.N, dtype=torch.float64, device=psi.device) if want_grad else None
        check(lib().llg_shape_penalty(self.h, _ptr(psi), float(xi), float(S_target), float(nu), float(x0), float(y0),
                                      _ptr(J), _ptr(g), _stream()))
        return J, g

    def shape_penalty_noalloc(self, psi, xi, S_target, nu, x0, y0, J, g=None):
        """shape_penalty into caller-provided J (1 double) and g (N doubles or
        None), through the entry point that allocates no device memory."""
        self._t(psi, self.N)
        check(lib().llg_shape_penalty_noalloc(self.h, _ptr(psi), float(xi), float(S_target), float(nu), float(x0),
                                              float(y0), _ptr(J), _ptr(g), _stream()))
        return J, g

    def field(self, psi, m, t=0.0, want_rhs=False):
        import torch
        self._t(psi, self.N)
        self._t(m, 3 * self.N)
        B = torch.empty(3 * self.N, dtype=self.tdtype, device=m.device)
        rhs = torch.empty_like(B) if want_rhs else None
        check(lib().llg_field(self.h, _ptr(psi), _ptr(m), float(t), _ptr(B), _ptr(rhs), _stream()))
        return (B, rhs) if want_rhs else B

    def forward(self, psi, m0, n_steps, t0=0.0, obj: Optional[Objective_c] = None, m_out=None):
        import torch
        self._t(psi, self.N)
        self._t(m0, 3 * self.N)
        _check_obj(obj, n_steps)
        m_out = torch.empty_like(m0) if m_out is None else m_out
        J = torch.zeros(1, dtype=torch.float64, device=m0.device)
        self._fwd_gen += 1
        check(lib().llg_forward(self.h, _ptr(psi), _ptr(m0), float(t0), int(n_steps),
                                ctypes.byref(obj) if obj is not None else None, _ptr(m_out), _ptr(J), _stream()))
        return m_out, J

    def objective(self, obj: Objective_c, psi, m, t=0.0):
        import torch
        dev = m.device
        J = torch.zeros(1, dtype=torch.float64, device=dev)
        dJdm = torch.empty(3 * self.N, dtype=self.tdtype, device=dev)
        dJdpsi = torch.empty(self.N, dtype=torch.float64, device=dev)
        en = torch.zeros(5, dtype=torch.float64, device=dev)
        check(lib().llg_objective(self.h, ctypes.byref(obj), _ptr(psi), _ptr(m), float(t), _ptr(J), _ptr(dJdm),
                                  _ptr(dJdpsi), _ptr(en), _stream()))
        return J, dJdm, dJdpsi, en

    def adjoint(self, psi, obj: Optional[Objective_c] = None, dJdm_T=None, dJdpsi_expl=None, want_dm0=False):
        import torch
        dev = psi.device
        dJdpsi = torch.empty(self.N, dtype=torch.float64, device=dev)
        dm0 = torch.empty(3 * self.N, dtype=self.tdtype, device=dev) if want_dm0 else None
        check(lib().llg_adjoint(self.h, _ptr(psi), _ptr(dJdm_T), _ptr(dJdpsi_expl),
                                ctypes.byref(obj) if obj is not None else None, _ptr(dJdpsi), _ptr(dm0), _stream()))
        return (dJdpsi, dm0) if want_dm0 else dJdpsi


def _parr(ts):
    """Host array of device pointers (None entries allowed)."""
    return (ctypes.c_void_p * len(ts))(*[None if t is None else t.data_ptr() for t in ts])


class Batch:
    """Many instances (designs x frequencies, ragged grids) integrated together;
    every kernel launch serves all of them (wraps llg_batch)."""

    def __init__(self, probs, dtype="f32", max_steps=1, masks=None, ckpt_policy=LLG_CKPT_SQRT, ckpt_param=0):
        import torch
        self.probs = list(probs)
        self.n = len(self.probs)
        self.dtype = dtype
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        self.N = [p.nx * p.ny * p.nz for p in self.probs]
        pcs = (Problem_c * self.n)(*[make_problem(p, dtype, max_steps, ckpt_policy, ckpt_param) for p in self.probs])
        keep = []
        mks = (Masks_c * self.n)()
        for i in range(self.n):
            mk = (masks or [{}] * self.n)[i] or {}
            vals = []
            for key in ("antenna", "port1", "port2", "design"):
                a = mk.get(key)
                if a is None:
                    vals.append(None)
                    continue
                arr = np.ascontiguousarray(np.asarray(a, dtype=np.uint8).reshape(-1))
                if arr.size != self.N[i]:
                    raise ValueError("mask size mismatch")
                keep.append(arr)
                vals.append(arr.ctypes.data)
            mks[i] = Masks_c(*vals)
        h = ctypes.c_void_p()
        check(lib().llg_batch_create(pcs, mks, self.n, ctypes.byref(h)))
        self.h = h
        self._fwd_gen = 0  # counts the forward records (forward, autotune) on this batch
        del keep

    def close(self):
        if getattr(self, "h", None):
            lib().llg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable, stride=1):
        """Event-time every stride-th launch of each kernel class while enable."""
        check(lib().llg_profile(self.h, int(stride) if enable else 0))

    def set_graphs(self, enable: bool):
        """Capture forward / adjoint launch sequences in HIP graphs and replay them."""
        check(lib().llg_set_graphs(self.h, int(enable)))

    def launch_config(self):
        """(column tile, column threads, column radix, forward row threads, forward radix,
        backward row threads, backward radix, staged values per row in the backward kernel)."""
        c = (ctypes.c_int32 * 8)()
        check(lib().llg_launch_config(self.h, c))
        return tuple(c)

    def set_launch_config(self, *cfg):
        """Eight values in the order of launch_config()."""
        c = (ctypes.c_int32 * 8)(*cfg)
        check(lib().llg_set_launch_config(self.h, c))

    def autotune(self):
        """Time the valid launch configurations and keep the fastest (drops the forward record)."""
        import torch
        check(lib().llg_autotune(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        self._fwd_gen += 1
        return self.launch_config()

    def profile_read(self, kind, reset=True):
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        check(lib().llg_profile_read(self.h, kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b), int(reset)))
        return ms.value, n.value, b.value

    def levelset_to_psi(self, phis, a, psi_fixed=None, extrude_z=True):
        import torch
        outs = [torch.empty(n, dtype=self.tdtype, device=phis[0].device) for n in self.N]
        pf = _parr(psi_fixed) if psi_fixed is not None else None
        check(lib().llg_batch_levelset_to_Ms(self.h, _parr(phis), pf, float(a), int(extrude_z), _parr(outs), _stream()))
        return outs

    def levelset_vjp(self, phis, dJdpsis, a, extrude_z=True):
        import torch
        outs = [torch.empty(p.numel(), dtype=torch.float64, device=p.device) for p in phis]
        check(lib().llg_batch_levelset_to_Ms_vjp(self.h, _parr(phis), _parr(dJdpsis), float(a), int(extrude_z),
                                                 _parr(outs), _stream()))
        return outs

    def forward(self, psis, m0s, n_steps, t0=0.0, obj: Optional[Objective_c] = None, want_m=True):
        import torch
        dev = psis[0].device
        _check_obj(obj, n_steps)
        m_out = [torch.empty(3 * n, dtype=self.tdtype, device=dev) for n in self.N] if want_m else None
        J = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self._fwd_gen += 1
        check(lib().llg_batch_forward(self.h, _parr(psis), _parr(m0s), float(t0), int(n_steps),
                                      ctypes.byref(obj) if obj is not None else None,
                                      _parr(m_out) if m_out is not None else None, ctypes.c_void_p(J.data_ptr()),
                                      _stream()))
        return m_out, J

    def adjoint(self, psis, obj: Optional[Objective_c] = None, dJdm_T=None, dJdpsi_expl=None, want_dm0=False):
        import torch
        dev = psis[0].device
        g = [torch.empty(n, dtype=torch.float64, device=dev) for n in self.N]
        dm0 = [torch.empty(3 * n, dtype=self.tdtype, device=dev) for n in self.N] if want_dm0 else None
        check(lib().llg_batch_adjoint(self.h, _parr(psis), _parr(dJdm_T) if dJdm_T is not None else None,
                                      _parr(dJdpsi_expl) if dJdpsi_expl is not None else None,
                                      ctypes.byref(obj) if obj is not None else None, _parr(g),
                                      _parr(dm0) if dm0 is not None else None, _stream()))
        return (g, dm0) if want_dm0 else g


class RBFLevelSet:
    """Level set from RBF amplitudes (Eqs. 2, 3 and the renormalisation after
    Eq. 3) on an nx x ny node grid: fixed centres (node units), c, p and design
    mask; the amplitudes s are the argument of each call (wraps
    llg_rbf_levelset / llg_rbf_levelset_vjp)."""

    def __init__(self, centers_x, centers_y, c, p, design, dtype="f32", normalize=True, device="cuda"):
        import torch
        D = np.asarray(design)
        if D.ndim != 2:
            raise ValueError("design must be a 2D (ny, nx) mask")
        self.ny, self.nx = D.shape
        xc = np.asarray(centers_x, np.float64).reshape(-1)
        yc = np.asarray(centers_y, np.float64).reshape(-1)
        if xc.shape != yc.shape or xc.size < 1:
            raise ValueError("centers_x and centers_y must have the same length >= 1")
        self.n = xc.size
        self.c, self.p, self.normalize = float(c), float(p), bool(normalize)
        self.dtype = LLG_F64 if dtype in ("f64", "float64", LLG_F64) else LLG_F32
        self.tdtype = torch.float64 if self.dtype == LLG_F64 else torch.float32
        self.device = torch.device(device)
        self.centers = torch.as_tensor(np.concatenate([xc, yc]), dtype=torch.float64, device=self.device)
        self.design = torch.as_tensor(np.ascontiguousarray(D != 0).astype(np.uint8).reshape(-1), device=self.device)
        v = ctypes.c_int64(0)
        check(lib().llg_rbf_work_len(self.nx, self.ny, self.n, ctypes.byref(v)))
        self.work_len = v.value

    def _s(self, s):
        import torch
        if s.dtype != torch.float64 or not s.is_cuda or not s.is_contiguous() or s.numel() != self.n:
            raise ValueError(f"expected a contiguous cuda tensor of {self.n} float64 amplitudes")
        return s

    def new_work(self):
        import torch
        return torch.empty(self.work_len, dtype=torch.float64, device=self.device)

    def levelset(self, s, want_pnorm=True, work=None):
        """(phi, pnorm, work): phi (nx*ny), the p-norm S for the VJP, and the
        workspace whose first two entries hold dphi and the scale."""
        import torch
        self._s(s)
        N = self.nx * self.ny
        phi = torch.empty(N, dtype=self.tdtype, device=self.device)
        pn = torch.empty(N, dtype=self.tdtype, device=self.device) if want_pnorm else None
        work = self.new_work() if work is None else work
        check(lib().llg_rbf_levelset(self.dtype, self.nx, self.ny, self.n, _ptr(self.centers), _ptr(s), self.c, self.p,
                                     _ptr(self.design), int(self.normalize), _ptr(phi), _ptr(pn), _ptr(work),
                                     _stream()))
        return phi, pn, work

    def vjp(self, s, dJdphi, pnorm, work):
        """dJ/ds (float64, n) from dJ/dphi (float64, nx*ny) and the pnorm and
        work of the levelset() call on the same s."""
        import torch
        self._s(s)
        if dJdphi.dtype != torch.float64 or dJdphi.numel() != self.nx * self.ny or not dJdphi.is_contiguous():
            raise ValueError("dJdphi must be a contiguous float64 tensor of nx*ny entries")
        if pnorm is None or pnorm.dtype != self.tdtype or pnorm.numel() != self.nx * self.ny:
            raise ValueError("pnorm must be the p-norm returned by levelset() for this s")
        if work is None or work.numel() != self.work_len:
            raise ValueError("work must be the workspace of the levelset() call")
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        check(lib().llg_rbf_levelset_vjp(self.dtype, self.nx, self.ny, self.n, _ptr(self.centers), _ptr(s), self.c,
                                         self.p, _ptr(self.design), _ptr(dJdphi), _ptr(pnorm), _ptr(work), _ptr(out),
                                         _stream()))
        return out


def rbf_profile(enable: bool):
    check(lib().llg_rbf_profile(int(enable)))


def rbf_profile_read(kind, reset=True):
    """(ms, launches, pairs) of one RBF pair kernel since the last reset."""
    ms, n, pr = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_double(0)
    check(lib().llg_rbf_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pr), int(reset)))
    return ms.value, n.value, pr.value


class Adam:
    """Adam moments of a float64 parameter vector on the device; step() updates
    it in place (wraps llg_adam_step)."""

    def __init__(self, n, lr, betas=(0.9, 0.999), eps=1e-8, device="cuda"):
        import torch
        self.lr, self.b1, self.b2, self.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        self.m = torch.zeros(n, dtype=torch.float64, device=device)
        self.v = torch.zeros(n, dtype=torch.float64, device=device)
        self.t = 0
        self.n = n

    def step(self, s, grad, lr=None):
        import torch
        for x in (s, grad):
            if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != self.n:
                raise ValueError(f"expected contiguous cuda float64 tensors of {self.n} entries")
        self.t += 1
        check(lib().llg_adam_step(self.n, _ptr(s), _ptr(grad), _ptr(self.m), _ptr(self.v), self.t,
                                  self.lr if lr is None else float(lr), self.b1, self.b2, self.eps, _stream()))
        return s
