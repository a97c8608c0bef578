"""Host checks of the autograd functions' wiring (no GPU): a stand-in solver
with the binding's method signatures and a small smooth map in place of the
LLG integration.  The functions must route every source and gradient to the
right call, scale by the incoming gradient and refuse a stale record; the
result is compared with torch autograd through the same map written directly.
The physics of the real path is tested on the GPU."""
import types

import pytest
import torch

from paper_2411_19109_amd import llg
from paper_2411_19109_amd.autograd import IntegrateLLG, LevelSet, LevelSetLLG, LLGObjective


class FakeSolver:
    """psi = tanh(a phi) + psi_fixed; m_T = m0 * n * psi (per component);
    port J = sum m_T^2; energy J = sum m_T^2 + sum psi."""

    def __init__(self, N, dtype=torch.float64):
        self.N = N
        self.tdtype = dtype
        self.prob = types.SimpleNamespace(dt=1e-13)
        self._fwd_gen = 0
        self._rec = None

    def levelset_to_psi(self, phi, a, psi_fixed=None, extrude_z=True):
        psi = torch.tanh(a * phi.double())
        return (psi if psi_fixed is None else psi + psi_fixed.double()).to(self.tdtype)

    def levelset_vjp(self, phi, g, a, extrude_z=True):
        t = torch.tanh(a * phi.double())
        return g.double() * a * (1 - t * t)

    def forward(self, psi, m0, n, t0=0.0, obj=None):
        self._fwd_gen += 1
        mT = m0 * n * psi.repeat(3)
        self._rec = (psi.clone(), m0.clone(), n)
        J = torch.zeros(1, dtype=torch.float64)
        if obj is not None and obj.kind == llg.LLG_OBJ_PORT_MY2:
            J += (mT.double() ** 2).sum()
        return mT, J

    def objective(self, obj, psi, m, t=0.0):
        J = ((m.double() ** 2).sum() + psi.double().sum()).reshape(1)
        return J, 2 * m, torch.ones(self.N, dtype=torch.float64), torch.zeros(5, dtype=torch.float64)

    def adjoint(self, psi, obj=None, dJdm_T=None, dJdpsi_expl=None, want_dm0=False):
        psi_r, m0, n = self._rec
        assert torch.equal(psi_r, psi)
        P = n * psi.repeat(3)
        lam = torch.zeros(3 * self.N, dtype=torch.float64)
        if dJdm_T is not None:
            lam += dJdm_T.double()
        if obj is not None and obj.kind == llg.LLG_OBJ_PORT_MY2:
            lam += 2 * (m0 * P).double()
        dpsi = (lam * m0.double() * n).reshape(3, -1).sum(0)
        if dJdpsi_expl is not None:
            dpsi += dJdpsi_expl
        dm0 = (lam * P.double()).to(self.tdtype)
        return (dpsi, dm0) if want_dm0 else dpsi


def _direct(phi, m0, a, pf, n, kind):
    psi = torch.tanh(a * phi) + pf
    mT = m0 * n * psi.repeat(3)
    J = (mT ** 2).sum()
    return J + psi.sum() if kind == llg.LLG_OBJ_ENERGY_AREA else J


@pytest.mark.parametrize("kind", [llg.LLG_OBJ_ENERGY_AREA, llg.LLG_OBJ_PORT_MY2])
def test_levelset_objective_wiring(kind):
    N, n, a = 7, 3, 0.8
    g = torch.Generator().manual_seed(3)
    phi0, m00, pf = (torch.randn(N, generator=g, dtype=torch.float64), torch.randn(3 * N, generator=g, dtype=torch.float64),
                     torch.rand(N, generator=g, dtype=torch.float64))
    obj = llg.make_objective(kind)
    ref_phi, ref_m0 = phi0.clone().requires_grad_(), m00.clone().requires_grad_()
    (-1.5 * _direct(ref_phi, ref_m0, a, pf, n, kind)).backward()
    for route in ("fused", "composed"):
        s = FakeSolver(N)
        phi, m0 = phi0.clone().requires_grad_(), m00.clone().requires_grad_()
        if route == "fused":
            J = LevelSetLLG.apply(phi, m0, s, obj, n, a, pf, True)
        else:
            J = LLGObjective.apply(LevelSet.apply(phi, s, a, pf, True), m0, s, obj, n)
        assert J.shape == ()
        assert torch.allclose(J, _direct(phi0, m00, a, pf, n, kind))
        (-1.5 * J).backward()
        assert torch.allclose(phi.grad, ref_phi.grad, rtol=1e-13), route
        assert torch.allclose(m0.grad, ref_m0.grad, rtol=1e-13), route


def test_integrate_wiring_and_stale_record():
    N, n = 5, 2
    g = torch.Generator().manual_seed(4)
    psi0, m00, w = (torch.rand(N, generator=g, dtype=torch.float64), torch.randn(3 * N, generator=g, dtype=torch.float64),
                    torch.randn(3 * N, generator=g, dtype=torch.float64))
    s = FakeSolver(N)
    psi, m0 = psi0.clone().requires_grad_(), m00.clone().requires_grad_()
    (w * IntegrateLLG.apply(psi, m0, s, n)).sum().backward()
    rp, rm = psi0.clone().requires_grad_(), m00.clone().requires_grad_()
    (w * (rm * n * rp.repeat(3))).sum().backward()
    assert torch.allclose(psi.grad, rp.grad) and torch.allclose(m0.grad, rm.grad)
    J = LLGObjective.apply(psi0.clone().requires_grad_(), m00, s, llg.make_objective(llg.LLG_OBJ_PORT_MY2), n)
    s.forward(psi0, m00, n)  # another trajectory recorded on the handle
    with pytest.raises(llg.LLGError):
        J.backward()
