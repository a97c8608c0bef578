"""torch.autograd functions over the forward/adjoint path.

The discrete adjoint of the RK4 map (the gradient of the discrete objective,
the discrete counterpart of the adjoint equations of Sec. 2, Eqs. 6-7) runs as
the backward of these functions, so a level-set design loop can be written as

    psi = LevelSet.apply(phi, solver, a, psi_fixed, True)
    J = LLGObjective.apply(psi, m0, solver, obj, n_steps)
    J.backward()                      # phi.grad = dJ/dphi

or, with the float64 chain from psi to phi kept inside the library,

    J = LevelSetLLG.apply(phi, m0, solver, obj, n_steps, a, psi_fixed, True)

and with the RBF amplitudes s as the design variables (Eqs. 2, 3), closing the
loop with an Adam step on s,

    phi = RBFLevelSetFn.apply(s, rbf)          # rbf: llg.RBFLevelSet
    J = LevelSetLLG.apply(phi, m0, solver, obj, n_steps, a, psi_fixed, True)
    J.backward(); adam.step(s.data, s.grad)    # adam: llg.Adam

and, for a batch of designs integrated together (one launch per stage for all),

    Js = BatchLevelSetLLG.apply(batch, obj, n_steps, a, psi_fixed_list, True, m0_list, *phis)

Marshalling only: forward and backward call the C ABI (``llg.Solver``,
``llg.Batch``), every step runs in the HIP library.  The adjoint walks the
checkpoints of the last forward on the handle, so a backward after another
forward on the same handle raises instead of returning a gradient of the wrong
trajectory.
"""
from __future__ import annotations

import torch

from . import llg


def _check_record(ctx):
    if ctx.solver._fwd_gen != ctx.gen:
        raise llg.LLGError(llg.LLG_ESTATE, "the handle ran another forward since this graph was built: "
                                           "the adjoint would walk the wrong trajectory")


def _terminal(solver, obj, psi, mT, t_end):
    """J and its terminal sources: the energy objective is evaluated at m_T;
    the port objective was accumulated during the forward."""
    if obj is not None and obj.kind == llg.LLG_OBJ_ENERGY_AREA:
        J, dJdm, dJdpsi_e, _ = solver.objective(obj, psi, mT, t=t_end)
        return J, dJdm, dJdpsi_e
    return None, None, None


class IntegrateLLG(torch.autograd.Function):
    """m_T = RK4^n(psi, m0) from t0 (Eq. 11, fixed step).  Backward: the adjoint
    started from lambda_N = dL/dm_T gives dL/dpsi and dL/dm0."""

    @staticmethod
    def forward(ctx, psi, m0, solver, n_steps, t0=0.0):
        mT, _ = solver.forward(psi.detach(), m0.detach(), n_steps, t0=t0)
        ctx.solver, ctx.gen = solver, solver._fwd_gen
        ctx.save_for_backward(psi)
        return mT

    @staticmethod
    def backward(ctx, g_mT):
        _check_record(ctx)
        (psi,) = ctx.saved_tensors
        s = ctx.solver
        src = g_mT.to(s.tdtype).contiguous()
        dpsi, dm0 = s.adjoint(psi.detach(), None, dJdm_T=src, want_dm0=True)
        return dpsi.to(psi.dtype), dm0, None, None, None


class LLGObjective(torch.autograd.Function):
    """J(psi, m0): the objective of the trajectory from m0 (energy-area at m_T,
    or the time-windowed port cost).  Backward: the adjoint with the
    objective's sources, scaled by the incoming gradient."""

    @staticmethod
    def forward(ctx, psi, m0, solver, obj, n_steps, t0=0.0):
        psi_d = psi.detach()
        mT, Jp = solver.forward(psi_d, m0.detach(), n_steps, t0=t0, obj=obj)
        J, dJdm, dJdpsi_e = _terminal(solver, obj, psi_d, mT, t0 + n_steps * solver.prob.dt)
        ctx.solver, ctx.gen, ctx.obj = solver, solver._fwd_gen, obj
        ctx.dJdm, ctx.dJdpsi_e = dJdm, dJdpsi_e
        ctx.save_for_backward(psi)
        return (Jp if J is None else J).reshape(())

    @staticmethod
    def backward(ctx, gJ):
        _check_record(ctx)
        (psi,) = ctx.saved_tensors
        dpsi, dm0 = ctx.solver.adjoint(psi.detach(), ctx.obj, dJdm_T=ctx.dJdm, dJdpsi_expl=ctx.dJdpsi_e,
                                       want_dm0=True)
        return (gJ * dpsi).to(psi.dtype), (gJ * dm0).to(dm0.dtype), None, None, None, None


class LevelSet(torch.autograd.Function):
    """psi = D * H(a phi) + (1 - D) * psi_fixed (Eq. 4 with the design mask),
    phi extruded through z when extrude_z.  Backward: the level-set VJP."""

    @staticmethod
    def forward(ctx, phi, solver, a, psi_fixed=None, extrude_z=True):
        psi = solver.levelset_to_psi(phi.detach(), a, psi_fixed, extrude_z)
        ctx.solver, ctx.a, ctx.extrude = solver, a, extrude_z
        ctx.save_for_backward(phi)
        return psi

    @staticmethod
    def backward(ctx, g_psi):
        (phi,) = ctx.saved_tensors
        dphi = ctx.solver.levelset_vjp(phi.detach(), g_psi.to(torch.float64).contiguous(), ctx.a, ctx.extrude)
        return dphi.to(phi.dtype), None, None, None, None


class LevelSetLLG(torch.autograd.Function):
    """J(phi, m0) in one function: level set, forward, objective; the backward
    keeps dJ/dpsi in float64 up to the level-set VJP."""

    @staticmethod
    def forward(ctx, phi, m0, solver, obj, n_steps, a, psi_fixed=None, extrude_z=True, t0=0.0):
        psi = solver.levelset_to_psi(phi.detach(), a, psi_fixed, extrude_z)
        mT, Jp = solver.forward(psi, m0.detach(), n_steps, t0=t0, obj=obj)
        J, dJdm, dJdpsi_e = _terminal(solver, obj, psi, mT, t0 + n_steps * solver.prob.dt)
        ctx.solver, ctx.gen, ctx.obj, ctx.a, ctx.extrude = solver, solver._fwd_gen, obj, a, extrude_z
        ctx.dJdm, ctx.dJdpsi_e, ctx.psi = dJdm, dJdpsi_e, psi
        ctx.save_for_backward(phi)
        return (Jp if J is None else J).reshape(())

    @staticmethod
    def backward(ctx, gJ):
        _check_record(ctx)
        (phi,) = ctx.saved_tensors
        s = ctx.solver
        dpsi, dm0 = s.adjoint(ctx.psi, ctx.obj, dJdm_T=ctx.dJdm, dJdpsi_expl=ctx.dJdpsi_e, want_dm0=True)
        dphi = s.levelset_vjp(phi.detach(), dpsi, ctx.a, ctx.extrude)
        return ((gJ * dphi).to(phi.dtype), (gJ * dm0).to(dm0.dtype), None, None, None, None, None, None, None)


class BatchLevelSetLLG(torch.autograd.Function):
    """J_i(phi_i) for every instance of an ``llg.Batch`` (port objective): one
    forward and one adjoint launch sequence serve all instances.  Returns the
    vector of J_i; the backward scales instance i's dJ_i/dphi_i by the incoming
    gradient's entry i."""

    @staticmethod
    def forward(ctx, batch, obj, n_steps, a, psi_fixed, extrude_z, m0s, *phis):
        if obj is None or obj.kind != llg.LLG_OBJ_PORT_MY2:
            raise llg.LLGError(llg.LLG_ENOTSUP, "batched objectives are running (port) costs")
        phis_d = [p.detach() for p in phis]
        psis = batch.levelset_to_psi(phis_d, a, psi_fixed, extrude_z)
        _, J = batch.forward(psis, [m.detach() for m in m0s], n_steps, obj=obj, want_m=False)
        ctx.batch, ctx.gen, ctx.obj, ctx.a, ctx.extrude, ctx.psis = batch, batch._fwd_gen, obj, a, extrude_z, psis
        ctx.save_for_backward(*phis)
        return J

    @staticmethod
    def backward(ctx, gJ):
        if ctx.batch._fwd_gen != ctx.gen:
            raise llg.LLGError(llg.LLG_ESTATE, "the batch ran another forward since this graph was built: "
                                               "the adjoint would walk the wrong trajectory")
        phis = ctx.saved_tensors
        b = ctx.batch
        dpsis = b.adjoint(ctx.psis, ctx.obj)
        dphis = b.levelset_vjp([p.detach() for p in phis], dpsis, ctx.a, ctx.extrude)
        return (None,) * 7 + tuple((gJ[i] * d).to(p.dtype) for i, (d, p) in enumerate(zip(dphis, phis)))


class RBFLevelSetFn(torch.autograd.Function):
    """phi(s): the renormalised p-norm of the RBF cones (Eqs. 2, 3), float64
    amplitudes in, phi in the RBF map's precision out.  Backward: dJ/ds with
    the shift and the renormalisation factor held at their forward values."""

    @staticmethod
    def forward(ctx, s, rbf):
        phi, pnorm, work = rbf.levelset(s.detach())
        ctx.rbf, ctx.pnorm, ctx.work = rbf, pnorm, work
        ctx.save_for_backward(s)
        return phi

    @staticmethod
    def backward(ctx, g_phi):
        (s,) = ctx.saved_tensors
        ds = ctx.rbf.vjp(s.detach(), g_phi.to(torch.float64).contiguous(), ctx.pnorm, ctx.work)
        return ds, None
