"""Magnetisation-curve objective (Eq. 8) with the linear field ramp through
the C ABI: J and dJ/dphi against the oracle (FP64 1e-9 / 1e-8, FP32 1e-3),
checkpoint policies and batching bitwise, argument checks, and the paper's
loop on the 30x30 particle (RBF level set, curve objective, Adam) against the
oracle chain."""
import numpy as np
import pytest

from _helpers import rel_l2, say, to_dev, to_np
from oracle import adjoint as oadj
from oracle import levelset as ols
from oracle import micromag as omm
from oracle import rbf as orbf
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu


def curve_case(n, nx=24, ny=20, seed=31, n_start=5):
    w = wl.sw_particle_curve(seed=seed, n_steps=n, nx=nx, ny=ny)
    w.problem.b_rf = (0.3, 0.0, 0.0)      # a steep ramp, so that M_x moves within a few dozen steps
    W = n - n_start
    w.obj_n_start = n_start
    tgt = np.linspace(0.02, 0.2, W)
    w.extra["target"], w.extra["weight"] = tgt, 1.0 / (tgt * W)
    return w


def gpu_curve(w, dtype, n, **kw):
    import torch
    from paper_2411_19109_amd import llg
    obj = llg.make_objective(wl.OBJ_MAG_CURVE, n_start=w.obj_n_start, target=w.extra["target"],
                             weight=w.extra["weight"])
    s = llg.Solver(w.problem, dtype=dtype, max_steps=n, antenna=w.antenna, design=w.design, **kw)
    phi = to_dev(w.phi, dtype)
    psi = s.levelset_to_psi(phi, w.heaviside_a, to_dev(w.psi_fixed, dtype))
    mT, J = s.forward(psi, to_dev(w.m0, dtype), n, obj=obj)
    dpsi, dm0 = s.adjoint(psi, obj, want_dm0=True)
    dphi = s.levelset_vjp(phi, dpsi, w.heaviside_a)
    torch.cuda.synchronize()
    out = dict(J=float(J.item()), dphi=to_np(dphi), dm0=to_np(dm0), mT=to_np(mT))
    s.close()
    return out


def oracle_curve(w, n):
    sim = omm.Sim(w.problem, antenna=w.antenna)
    psi = ols.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    obj = oadj.Objective(oadj.OBJ_MAG_CURVE, n_start=w.obj_n_start, target=w.extra["target"],
                         weight=w.extra["weight"])
    J, gpsi, lam0 = oadj.gradient(sim, w.m0, psi, n, obj)
    return J, ols.levelset_vjp(w.phi, w.heaviside_a, w.design, gpsi).reshape(-1), lam0.reshape(-1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_curve_gradient_matches_oracle(dtype):
    n = 30
    w = curve_case(n)
    say("curve objective, field ramp,", n, "steps", dtype)
    g = gpu_curve(w, dtype, n, ckpt_param=4)
    Jo, go, lo = oracle_curve(w, n)
    say("  J gpu / oracle", g["J"], Jo, "dJ/dphi rel L2", rel_l2(g["dphi"], go), "dJ/dm0", rel_l2(g["dm0"], lo))
    if dtype == "f64":
        assert abs(g["J"] - Jo) <= 1e-10 * abs(Jo)
        assert rel_l2(g["dphi"], go) <= 1e-9
        assert rel_l2(g["dm0"], lo) <= 1e-9
    else:
        assert abs(g["J"] - Jo) <= 1e-4 * abs(Jo)
        assert rel_l2(g["dphi"], go) <= 1e-3
        assert rel_l2(g["dm0"], lo) <= 1e-3


def test_curve_gradient_is_the_same_under_every_checkpoint_policy_and_in_a_batch():
    import torch
    from paper_2411_19109_amd import llg
    n = 24
    w = curve_case(n, seed=32)
    a = gpu_curve(w, "f64", n, ckpt_policy=llg.LLG_CKPT_SQRT, ckpt_param=4)
    b = gpu_curve(w, "f64", n, ckpt_policy=llg.LLG_CKPT_ALL)
    c = gpu_curve(w, "f64", n, ckpt_policy=llg.LLG_CKPT_BINOMIAL, ckpt_param=3)
    assert a["J"] == b["J"] == c["J"]
    assert np.array_equal(a["dphi"], b["dphi"]) and np.array_equal(a["dphi"], c["dphi"])
    ws = [curve_case(n, nx=24, ny=20, seed=33), curve_case(n, nx=18, ny=26, seed=34)]
    obj = llg.make_objective(wl.OBJ_MAG_CURVE, n_start=ws[0].obj_n_start, target=ws[0].extra["target"],
                             weight=ws[0].extra["weight"])
    for w2 in ws[1:]:
        w2.extra["target"], w2.extra["weight"] = ws[0].extra["target"], ws[0].extra["weight"]
    bt = llg.Batch([x.problem for x in ws], dtype="f32", max_steps=n,
                   masks=[dict(antenna=x.antenna, design=x.design) for x in ws])
    phis = [to_dev(x.phi, "f32") for x in ws]
    psis = bt.levelset_to_psi(phis, ws[0].heaviside_a, [to_dev(x.psi_fixed, "f32") for x in ws])
    _, J = bt.forward(psis, [to_dev(x.m0, "f32") for x in ws], n, obj=obj)
    gg = bt.adjoint(psis, obj)
    dphi = bt.levelset_vjp(phis, gg, ws[0].heaviside_a)
    torch.cuda.synchronize()
    for i, x in enumerate(ws):
        so = gpu_curve(x, "f32", n)
        assert float(J[i].item()) == so["J"], i
        assert np.array_equal(to_np(dphi[i]), so["dphi"]), i
    bt.close()


def test_curve_objective_argument_checks():
    from paper_2411_19109_amd import llg
    n = 10
    w = curve_case(n, n_start=2)
    s = llg.Solver(w.problem, dtype="f32", max_steps=n, antenna=w.antenna, design=w.design)
    psi = to_dev(np.ones(w.problem.n), "f32")
    short = llg.make_objective(wl.OBJ_MAG_CURVE, n_start=2, target=np.ones(3), weight=np.ones(3))
    with pytest.raises(ValueError):
        s.forward(psi, to_dev(w.m0, "f32"), n, obj=short)
    bad = w.extra["target"].copy()
    bad[1] = np.nan
    with pytest.raises(llg.LLGError):
        s.forward(psi, to_dev(w.m0, "f32"), n, obj=llg.make_objective(wl.OBJ_MAG_CURVE, n_start=2, target=bad,
                                                                       weight=w.extra["weight"]))
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_particle_curve_design_loop_matches_oracle(dtype):
    """The paper's first task on its 30x30 particle (3 nm cells, ramp to 0.3 Ms
    along x, 20x20 RBFs over the mesh), on a 40-step prefix: s -> phi -> psi ->
    J (Eq. 8) and dJ/ds through the autograd functions, then an Adam step,
    twice, each against the oracle chain at the current s."""
    import torch
    from paper_2411_19109_amd import llg
    from paper_2411_19109_amd.autograd import LevelSetLLG, RBFLevelSetFn
    n = 40
    w = wl.sw_particle_curve(n_steps=n)
    lay = w.extra["rbf"]
    D2 = w.design[0]
    rbfm = llg.RBFLevelSet(lay["xc"], lay["yc"], lay["c"], lay["p"], D2, dtype=dtype)
    solver = llg.Solver(w.problem, dtype=dtype, max_steps=n, antenna=w.antenna, design=w.design)
    obj = llg.make_objective(wl.OBJ_MAG_CURVE, n_start=0, target=w.extra["target"], weight=w.extra["weight"])
    s = torch.as_tensor(lay["s"], dtype=torch.float64, device="cuda").requires_grad_()
    opt = llg.Adam(s.numel(), lr=0.05)
    o_obj = oadj.Objective(oadj.OBJ_MAG_CURVE, n_start=0, target=w.extra["target"], weight=w.extra["weight"])
    sim = omm.Sim(w.problem, antenna=w.antenna)
    ctr = (lay["xc"], lay["yc"])
    for t in range(1, 3):
        s.grad = None
        phi = RBFLevelSetFn.apply(s, rbfm)
        J = LevelSetLLG.apply(phi, to_dev(w.m0, dtype), solver, obj, n, w.heaviside_a, to_dev(w.psi_fixed, dtype),
                              True)
        J.backward()
        torch.cuda.synchronize()
        s_now, g_now = to_np(s.detach()), to_np(s.grad)
        ophi, od, osc = orbf.pnorm_levelset(s_now, ctr, lay["c"], lay["p"], D2)
        psi = ols.levelset_to_psi(ophi, w.heaviside_a, w.design, w.psi_fixed)
        Jo, gpsi, _ = oadj.gradient(sim, w.m0, psi, n, o_obj)
        gphi = ols.levelset_vjp(ophi, w.heaviside_a, w.design, gpsi)
        dso = orbf.pnorm_levelset_vjp(s_now, ctr, lay["c"], lay["p"], D2, gphi, od, osc)
        say("curve design step", t, dtype, "J", float(J.item()), Jo, "dJ/ds rel L2", rel_l2(g_now, dso))
        assert abs(float(J.item()) - Jo) <= (1e-10 if dtype == "f64" else 1e-4) * abs(Jo)
        assert rel_l2(g_now, dso) <= (1e-8 if dtype == "f64" else 1e-3)
        opt.step(s.data, s.grad)
    solver.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nz", [1, 2])
def test_shape_constraints_match_oracle(dtype, nz):
    import torch
    from oracle import shape as oshape
    from paper_2411_19109_amd import llg
    p = wl.Problem(nx=37, ny=29, nz=nz, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5, A=1.3e-11, terms=wl.TERM_EXCH)
    rng = np.random.default_rng(40 + nz)
    psi = rng.uniform(0.0, 1.0, p.shape) ** 3
    s = llg.Solver(p, dtype=dtype, max_steps=1)
    args = (0.05, 120.0, 1.0, 17.0, 11.5)
    J, g = s.shape_penalty(to_dev(psi, dtype), *args)
    torch.cuda.synchronize()
    psi_used = to_np(to_dev(psi, dtype)).reshape(p.shape)   # the values the GPU saw
    Jo = oshape.penalty(psi_used, *args)
    go = oshape.penalty_grad(psi_used, *args).reshape(-1)
    say("shape constraints", dtype, nz, "J", float(J.item()), Jo)
    assert abs(float(J.item()) - Jo) <= 1e-12 * abs(Jo)
    assert rel_l2(to_np(g), go) <= 1e-12
    s.close()


def test_regularised_objective_gradient_matches_oracle():
    """Eq. 9: zeta x the curve term + the size and centre constraints, the
    constraint gradient passed to the adjoint as its explicit dJ/dpsi."""
    import torch
    from oracle import shape as oshape
    from paper_2411_19109_amd import llg
    n, zeta = 24, 10.0
    w = curve_case(n, seed=35)
    psi_o = ols.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    # targets near the map's own area and centre, so that no term swamps the others
    args = (0.05, psi_o.sum() - 2.0, 1.0, 11.0, 9.0)
    tgt, wt = w.extra["target"], zeta * w.extra["weight"]
    obj = llg.make_objective(wl.OBJ_MAG_CURVE, n_start=w.obj_n_start, target=tgt, weight=wt)
    s = llg.Solver(w.problem, dtype="f64", max_steps=n, antenna=w.antenna, design=w.design)
    phi = to_dev(w.phi, "f64")
    psi = s.levelset_to_psi(phi, w.heaviside_a, to_dev(w.psi_fixed, "f64"))
    _, Jc = s.forward(psi, to_dev(w.m0, "f64"), n, obj=obj)
    Js, gs = s.shape_penalty(psi, *args)
    dpsi = s.adjoint(psi, obj, dJdpsi_expl=gs)
    dphi = s.levelset_vjp(phi, dpsi, w.heaviside_a)
    torch.cuda.synchronize()
    J = float(Jc.item()) + float(Js.item())
    sim = omm.Sim(w.problem, antenna=w.antenna)
    o = oadj.Objective(oadj.OBJ_MAG_CURVE, n_start=w.obj_n_start, target=tgt, weight=wt)
    Jo, gpsi, _ = oadj.gradient(sim, w.m0, psi_o, n, o)
    Jo += oshape.penalty(psi_o, *args)
    gpsi = gpsi + oshape.penalty_grad(psi_o, *args)
    go = ols.levelset_vjp(w.phi, w.heaviside_a, w.design, gpsi).reshape(-1)
    say("Eq. 9 J", J, Jo, "(curve", float(Jc.item()), ") dJ/dphi rel L2", rel_l2(to_np(dphi), go))
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert rel_l2(to_np(dphi), go) <= 1e-9
    s.close()
