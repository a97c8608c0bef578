"""Shared helpers of the GPU parity tests: build both sides from one workload."""
import sys

import numpy as np

from oracle import adjoint as oadj
from oracle import levelset as ols
from oracle import micromag as omm
from paper_2411_19109_amd import workloads as wl


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float64)).reshape(-1), dtype=td, device=torch_dev())


def to_np(t, shape=None):
    a = t.detach().to("cpu").double().numpy()
    return a.reshape(shape) if shape is not None else a


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_objective(w, kind=None):
    kind = w.objective if kind is None else kind
    return oadj.Objective(kind, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area,
                          n_start=w.obj_n_start, port1=w.port1, port2=w.port2)


def oracle_psi(w):
    return ols.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)


def oracle_sim(w):
    return omm.Sim(w.problem, antenna=w.antenna)


def gpu_solver(w, dtype=None, max_steps=None, tune=False, **kw):
    """A handle for the workload; tune=True runs the autotuner (the benchmark's setup)."""
    from paper_2411_19109_amd import llg
    s = llg.Solver(w.problem, dtype=dtype or w.dtype, max_steps=max_steps or w.n_steps, antenna=w.antenna,
                   port1=w.port1, port2=w.port2, design=w.design, **kw)
    if tune:
        say("autotuned launch", s.autotune())
    return s


def gpu_objective(w, kind=None):
    from paper_2411_19109_amd import llg
    kind = w.objective if kind is None else kind
    return llg.make_objective(kind, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area,
                              n_start=w.obj_n_start)


def gpu_gradient(w, dtype, n_steps=None, kind=None, solver=None, **kw):
    """J, dJ/dphi (extruded phi), dJ/dpsi and dJ/dm0 through the C ABI."""
    import torch
    n = n_steps or w.n_steps
    kind = w.objective if kind is None else kind
    s = solver or gpu_solver(w, dtype, max_steps=n, **kw)
    phi = to_dev(w.phi, dtype)
    psi = s.levelset_to_psi(phi, w.heaviside_a, to_dev(w.psi_fixed, dtype), extrude_z=True)
    m0 = to_dev(w.m0, dtype)
    obj = gpu_objective(w, kind)
    mT, Jp = s.forward(psi, m0, n, obj=obj)
    if kind == wl.OBJ_ENERGY_AREA:
        J, dJdm, dJdpsi_e, _ = s.objective(obj, psi, mT)
    else:
        J, dJdm, dJdpsi_e = Jp, None, None
    dJdpsi, dm0 = s.adjoint(psi, obj, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, want_dm0=True)
    dJdphi = s.levelset_vjp(phi, dJdpsi, w.heaviside_a, extrude_z=True)
    torch.cuda.synchronize()
    return dict(J=float(J.item()), dphi=to_np(dJdphi), dpsi=to_np(dJdpsi), dm0=to_np(dm0), mT=to_np(mT), solver=s)


def oracle_gradient(w, n_steps=None, kind=None):
    n = n_steps or w.n_steps
    sim = oracle_sim(w)
    psi = oracle_psi(w)
    obj = oracle_objective(w, kind)
    J, gpsi, lam0 = oadj.gradient(sim, w.m0, psi, n, obj)
    gphi = ols.levelset_vjp(w.phi, w.heaviside_a, w.design, gpsi)
    return dict(J=J, dphi=gphi.reshape(-1), dpsi=gpsi.reshape(-1), dm0=lam0.reshape(-1))
