"""Adaptive Dormand-Prince integration and the adjoint of its accepted steps
through the C ABI: the accepted step sequence, m(t_end), J and dJ/dphi against
the oracle's adaptive run (FP64 1e-10 / 1e-9), FP32 against the oracle replay
of the GPU's own steps, rejected trials, call-order checks, and bitwise-equal
results with the optional stage store."""
import numpy as np
import pytest

from _helpers import rel_l2, rel_max, say, to_dev, to_np
from oracle import adjoint as oadj
from oracle import dopri as odp
from oracle import levelset as ols
from oracle import micromag as omm
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu


def case(nx=12, ny=9, seed=51, terms=wl.TERM_ALL):
    p = wl.Problem(nx=nx, ny=ny, nz=1, dx=3e-9, dy=3e-9, dz=4e-9, Ms=8e5, A=1.3e-11, K=5e4, ku=(0.6, 0.8, 0.0),
                   alpha0=0.2, alpha_max=0.2, B0=(0.05, 0.02, 0.1), b_rf=(0.0, 0.01, 0.0), f1=5e9,
                   terms=terms, dt=5e-14)
    rng = np.random.default_rng(seed)
    sh = p.shape
    ant = np.zeros(sh, np.uint8)
    ant[:, :, 1] = 1
    phi = rng.standard_normal((ny, nx)) * 0.5
    design = np.ones(sh, np.uint8)
    psif = np.zeros(sh)
    m0 = rng.standard_normal((3,) + sh)
    m0 /= np.sqrt((m0 ** 2).sum(0))
    return p, ant, phi, design, psif, m0


def gpu_run(dtype, t_end, h0, tol, seed=51, terms=wl.TERM_ALL):
    import torch
    from paper_2411_19109_amd import llg
    p, ant, phi, design, psif, m0 = case(seed=seed, terms=terms)
    s = llg.Solver(p, dtype=dtype, max_steps=400, antenna=ant, design=design)
    ph = to_dev(phi, dtype)
    psi = s.levelset_to_psi(ph, 3.0, to_dev(psif, dtype))
    mT, hs, nrej = s.forward_adaptive(psi, to_dev(m0, dtype), t_end, h0, tol, tol)
    obj = llg.make_objective(wl.OBJ_ENERGY_AREA, E_ref=1e-18, lam=0.7, area=0.4)
    J, dJdm, dJdpsi_e, _ = s.objective(obj, psi, mT)
    dpsi, dm0 = s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, want_dm0=True)
    dphi = s.levelset_vjp(ph, dpsi, 3.0)
    torch.cuda.synchronize()
    out = dict(mT=to_np(mT), hs=np.asarray(hs), nrej=nrej, J=float(J.item()), dphi=to_np(dphi), dm0=to_np(dm0))
    s.close()
    return out


def oracle_replay(hs, seed=51, terms=wl.TERM_ALL):
    p, ant, phi, design, psif, m0 = case(seed=seed, terms=terms)
    sim = omm.Sim(p, antenna=ant)
    psi = ols.levelset_to_psi(phi, 3.0, design, psif)
    obj = oadj.Objective(oadj.OBJ_ENERGY_AREA, E_ref=1e-18, lam=0.7, area=0.4)
    mT = odp.integrate_fixed(sim, m0, psi, 0.0, list(hs))
    J, gpsi, lam0 = odp.gradient_fixed(sim, m0, psi, 0.0, list(hs), obj)
    return dict(mT=mT.reshape(-1), J=J, dphi=ols.levelset_vjp(phi, 3.0, design, gpsi).reshape(-1), dm0=lam0.reshape(-1),
                sim=sim, psi=psi, m0=m0)


def test_adaptive_run_and_gradient_match_oracle_fp64():
    t_end, h0, tol = 3e-12, 2e-13, 1e-7
    g = gpu_run("f64", t_end, h0, tol)
    o = oracle_replay(g["hs"])
    _, hs_o, rej_o = odp.integrate_adaptive(o["sim"], o["m0"], o["psi"], 0.0, t_end, h0, tol, tol)
    say("adaptive f64:", len(g["hs"]), "steps,", g["nrej"], "rejected; oracle", len(hs_o), rej_o)
    assert len(g["hs"]) == len(hs_o) and g["nrej"] == rej_o
    # the error estimate is a difference of nearly equal stage sums: its relative rounding is far above the
    # state's, and the next step follows it to the power -1/5; the sequences agree to that level (the state
    # and the gradient are compared on the GPU's own steps)
    say("  step sizes: max relative difference", np.abs(g["hs"] / np.asarray(hs_o) - 1).max())
    assert np.allclose(g["hs"], hs_o, rtol=1e-6, atol=0)
    assert g["nrej"] >= 1 and len(set(np.round(g["hs"] / 1e-16))) > 1
    assert rel_max(g["mT"], o["mT"]) <= 1e-10
    assert abs(g["J"] - o["J"]) <= 1e-10 * abs(o["J"])
    say("  dJ/dphi rel L2", rel_l2(g["dphi"], o["dphi"]), "dJ/dm0", rel_l2(g["dm0"], o["dm0"]))
    assert rel_l2(g["dphi"], o["dphi"]) <= 1e-9
    assert rel_l2(g["dm0"], o["dm0"]) <= 1e-9


def test_adaptive_fp32_matches_oracle_replay_of_its_steps():
    g = gpu_run("f32", 3e-12, 2e-13, 1e-4)
    o = oracle_replay(g["hs"])
    say("adaptive f32:", len(g["hs"]), "steps; m max err", np.abs(g["mT"] - o["mT"]).max(),
        "dJ/dphi rel L2", rel_l2(g["dphi"], o["dphi"]))
    assert np.abs(g["mT"] - o["mT"]).max() <= 1e-4
    assert abs(g["J"] - o["J"]) <= 1e-3 * abs(o["J"])
    assert rel_l2(g["dphi"], o["dphi"]) <= 1e-3


def test_adaptive_without_demag_matches_oracle_fp64():
    """Exchange, Zeeman with drive and anisotropy only: the field evaluations
    have no transforms, and each stage's state sum stands alone in the launch."""
    terms = wl.TERM_EXCH | wl.TERM_ZEEMAN | wl.TERM_ANIS
    g = gpu_run("f64", 3e-12, 2e-13, 1e-7, terms=terms)
    o = oracle_replay(g["hs"], terms=terms)
    _, hs_o, rej_o = odp.integrate_adaptive(o["sim"], o["m0"], o["psi"], 0.0, 3e-12, 2e-13, 1e-7, 1e-7)
    say("adaptive f64 without demag:", len(g["hs"]), "steps,", g["nrej"], "rejected; dJ/dphi rel L2",
        rel_l2(g["dphi"], o["dphi"]))
    assert len(g["hs"]) == len(hs_o) and g["nrej"] == rej_o
    assert np.allclose(g["hs"], hs_o, rtol=1e-6, atol=0)
    assert rel_max(g["mT"], o["mT"]) <= 1e-10
    assert rel_l2(g["dphi"], o["dphi"]) <= 1e-9
    assert rel_l2(g["dm0"], o["dm0"]) <= 1e-9


def test_adaptive_call_checks():
    import torch
    from paper_2411_19109_amd import llg
    p, ant, phi, design, psif, m0 = case()
    s = llg.Solver(p, dtype="f64", max_steps=400, antenna=ant, design=design)
    psi = to_dev(np.ones(p.n), "f64")
    with pytest.raises(llg.LLGError):
        s.adjoint_adaptive(psi)
    with pytest.raises(llg.LLGError):
        s.forward_adaptive(psi, to_dev(m0, "f64"), -1e-12, 1e-13, 1e-6, 1e-6)
    small = llg.Solver(p, dtype="f64", max_steps=3, antenna=ant, design=design)
    with pytest.raises(llg.LLGError):
        small.forward_adaptive(psi, to_dev(m0, "f64"), 3e-12, 1e-13, 1e-6, 1e-6)
    torch.cuda.synchronize()
    small.close()
    s.close()


@pytest.mark.parametrize("dtype,tol,terms", [("f64", 1e-7, wl.TERM_ALL), ("f32", 1e-4, wl.TERM_ALL),
                                              ("f32", 1e-4, wl.TERM_EXCH | wl.TERM_ZEEMAN | wl.TERM_ANIS)])
def test_kept_stages_give_bitwise_the_same_gradient(dtype, tol, terms):
    """With the stage store the adjoint reads the forward's stage states and
    fields instead of recomputing them: the same accepted steps, m(t_end),
    dJ/dpsi and dJ/dm0, bit for bit (runs with rejected trials included); the
    store stays valid for the run that filled it."""
    import torch
    from paper_2411_19109_amd import llg
    p, ant, phi, design, psif, m0 = case(terms=terms)
    out = {}
    for keep in (False, True):
        s = llg.Solver(p, dtype=dtype, max_steps=400, antenna=ant, design=design)
        s.set_keep_stages(keep)
        ph = to_dev(phi, dtype)
        psi = s.levelset_to_psi(ph, 3.0, to_dev(psif, dtype))
        # an oversized first step (1 ps) is rejected, so rejected trials write into the store too
        mT, hs, nrej = s.forward_adaptive(psi, to_dev(m0, dtype), 3e-12, 1e-12, tol, tol)
        obj = llg.make_objective(wl.OBJ_ENERGY_AREA, E_ref=1e-18, lam=0.7, area=0.4)
        _, dJdm, dJdpsi_e, _ = s.objective(obj, psi, mT)
        dpsi, dm0 = s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, want_dm0=True)
        if keep:
            s.set_keep_stages(False)   # the store of the last run is still read
            dpsi2, dm02 = s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, want_dm0=True)
            np.testing.assert_array_equal(to_np(dpsi2), to_np(dpsi))
            np.testing.assert_array_equal(to_np(dm02), to_np(dm0))
        torch.cuda.synchronize()
        out[keep] = (np.asarray(hs), nrej, to_np(mT), to_np(dpsi), to_np(dm0))
        s.close()
    say(f"kept stages {dtype}: {len(out[True][0])} steps, {out[True][1]} rejected")
    assert out[True][1] >= 1
    for a, b in zip(out[False], out[True]):
        np.testing.assert_array_equal(a, b)
