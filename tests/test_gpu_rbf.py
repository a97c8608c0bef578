"""RBF level set (Eqs. 2, 3, renormalisation), its VJP and the Adam update
through the C ABI, against the float64 oracle (oracle/rbf.py).

Tolerances: FP64 1e-10 relative max-norm for phi, the p-norm, the shift and
the scale, 1e-10 relative L2 for dJ/ds; FP32 phi within 2e-5 of max |phi| (1
once phi is renormalised into [-1, 1]; each power (b/S)^p carries about p ulps of relative
error, and the p-th root takes it back to a few ulps of S, which is of order
the shift, tens of nodes), FP32 dJ/ds within 1e-3 relative L2."""
import numpy as np
import pytest

from _helpers import oracle_gradient, rel_l2, rel_max, say, to_dev, to_np
from oracle import rbf as orbf
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_PHI = {"f64": 1e-10, "f32": 2e-5}
TOL_GRAD = {"f64": 1e-10, "f32": 1e-3}


def box_design(nx, ny, box):
    x0, y0, D = box
    d = np.zeros((ny, nx), np.uint8)
    d[y0:y0 + D, x0:x0 + D] = 1
    return d


def gpu_map(lay, design, dtype, normalize=True):
    from paper_2411_19109_amd import llg
    return llg.RBFLevelSet(lay["xc"], lay["yc"], lay["c"], lay["p"], design, dtype=dtype, normalize=normalize)


def s_dev(s):
    import torch
    return torch.as_tensor(np.asarray(s, np.float64), device="cuda")


def run_pair(lay, design, dtype, normalize=True, seed=0):
    """GPU and oracle phi, p-norm, shift, scale and dJ/ds for a random dJ/dphi."""
    import torch
    m = gpu_map(lay, design, dtype, normalize)
    s = s_dev(lay["s"])
    phi, pn, work = m.levelset(s)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(design.shape) * design
    ds = m.vjp(s, to_dev(w, "f64"), pn, work)
    torch.cuda.synchronize()
    ctr = (lay["xc"], lay["yc"])
    ophi, od, osc = orbf.pnorm_levelset(lay["s"], ctr, lay["c"], lay["p"], design, normalize=normalize)
    oraw, _, _ = orbf.pnorm_levelset(lay["s"], ctr, lay["c"], lay["p"], design, normalize=False)
    ods = orbf.pnorm_levelset_vjp(lay["s"], ctr, lay["c"], lay["p"], design, w, od, osc)
    D = design.astype(bool).reshape(-1)
    wk = to_np(work)
    return dict(phi=to_np(phi), pn=to_np(pn), dphi=wk[0], scale=wk[1], ds=to_np(ds),
                ophi=ophi.reshape(-1), opn=(oraw.reshape(-1) + od) * D, odphi=od, oscale=osc, ods=ods, D=D)


def check(r, dtype):
    D = r["D"]
    say("  phi max err", np.abs(r["phi"] - r["ophi"]).max(), "dJ/ds rel L2", rel_l2(r["ds"], r["ods"]))
    assert np.all(r["phi"][~D] == 0)
    if dtype == "f64":
        assert rel_max(r["phi"], r["ophi"]) <= TOL_PHI["f64"]
        assert rel_max(r["pn"][D], r["opn"][D]) <= 1e-10
    else:
        assert np.abs(r["phi"] - r["ophi"]).max() <= TOL_PHI["f32"] * max(1.0, np.abs(r["ophi"]).max())
    assert abs(r["dphi"] - r["odphi"]) <= (1e-12 if dtype == "f64" else 1e-5) * max(1.0, r["odphi"])
    assert abs(r["scale"] - r["oscale"]) <= (1e-10 if dtype == "f64" else 1e-5) * r["oscale"]
    assert rel_l2(r["ds"], r["ods"]) <= TOL_GRAD[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_demux_design_region_matches_oracle(dtype):
    """The demultiplexer's 60x60 design square in its 256x96 grid, 20x20 RBFs
    with a 4x4 grid of holes (the paper's configuration)."""
    w = wl.yig_demux(n_steps=10)
    lay = wl.rbf_layout(w.extra["box"], holes=4, seed=1)
    say("rbf demux 256x96, 400 RBFs", dtype)
    r = run_pair(lay, w.design[0], dtype)
    check(r, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny,n_side", [(64, 64, 20), (300, 200, 7), (400, 375, 5), (517, 509, 6), (37, 23, 39)])
def test_grid_sizes_and_rbf_counts(dtype, nx, ny, n_side):
    """Sizes that select the lanes-per-node splits 16, 8, 2 and 1 (small grids
    split a node's RBFs over more lanes), ragged last blocks, and 1521 RBFs
    (two LDS chunks, the second ragged)."""
    D = min(nx, ny) - 2
    box = (1, 1, D)
    lay = wl.rbf_layout(box, n_side=n_side, holes=2, seed=nx)
    design = box_design(nx, ny, box)
    say("rbf", nx, "x", ny, n_side * n_side, "RBFs", dtype)
    check(run_pair(lay, design, dtype, seed=ny), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("p", [1.0, 2.0, 7.5])
def test_other_norm_orders(dtype, p):
    """p = 1 (the sum, where the VJP's exponent p - 1 vanishes), p = 2 and a
    non-integer p, without renormalisation."""
    lay = wl.rbf_layout((3, 2, 30), n_side=6, holes=1, seed=3, p=p)
    design = box_design(40, 36, (3, 2, 30))
    say("rbf p =", p, dtype)
    check(run_pair(lay, design, dtype, normalize=False), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_rbf_and_single_node(dtype):
    lay = dict(xc=np.array([5.25]), yc=np.array([3.5]), c=1.5, p=90.0, s=np.array([4.0]))
    design = np.ones((9, 12), np.uint8)
    say("rbf single cone", dtype)
    check(run_pair(lay, design, dtype), dtype)
    for s0 in (-3.0, 3.0):
        # one node, one cone g: phi = g renormalised to sign(g); for g < 0 the
        # only base is 0 (the p-norm's kink) and dJ/ds = 0 on both sides
        lay1 = dict(xc=np.array([0.3]), yc=np.array([0.0]), c=1.0, p=90.0, s=np.array([s0]))
        r = run_pair(lay1, np.ones((1, 1), np.uint8), dtype)
        assert r["phi"][0] == pytest.approx(np.sign(s0), abs=1e-6)
        if s0 < 0:
            assert r["ds"][0] == 0 and r["ods"][0] == 0
        else:
            check(r, dtype)


def test_empty_design_region_gives_zero_phi_and_gradient():
    import torch
    lay = wl.rbf_layout((0, 0, 16), n_side=4, holes=0, seed=0)
    design = np.zeros((16, 16), np.uint8)
    m = gpu_map(lay, design, "f32")
    s = s_dev(lay["s"])
    phi, pn, work = m.levelset(s)
    ds = m.vjp(s, to_dev(np.ones((16, 16)), "f64"), pn, work)
    torch.cuda.synchronize()
    assert np.all(to_np(phi) == 0) and np.all(to_np(ds) == 0)
    assert to_np(work)[0] == 0 and to_np(work)[1] == 1


def test_repeated_calls_are_bitwise_identical():
    import torch
    w = wl.yig_demux(n_steps=10)
    lay = wl.rbf_layout(w.extra["box"], holes=4, seed=2)
    m = gpu_map(lay, w.design[0], "f32")
    s = s_dev(lay["s"])
    g = to_dev(np.random.default_rng(1).standard_normal(w.design[0].shape), "f64")
    outs = []
    for _ in range(3):
        phi, pn, work = m.levelset(s)
        outs.append((to_np(phi), to_np(m.vjp(s, g, pn, work))))
    torch.cuda.synchronize()
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])


def test_adam_matches_oracle_over_steps():
    import torch
    from paper_2411_19109_amd import llg
    rng = np.random.default_rng(4)
    n = 1000
    s = rng.standard_normal(n)
    grads = rng.standard_normal((6, n)) * np.logspace(-4, 2, n)
    opt = llg.Adam(n, lr=0.03)
    sd = s_dev(s)
    m = v = np.zeros(n)
    so = s.copy()
    for t in range(1, 7):
        opt.step(sd, s_dev(grads[t - 1]))
        so, m, v = orbf.adam_step(so, grads[t - 1], m, v, t, lr=0.03)
    torch.cuda.synchronize()
    assert rel_max(to_np(sd), so) <= 1e-13
    assert rel_max(to_np(opt.m), m) <= 1e-13 and rel_max(to_np(opt.v), v) <= 1e-13


def particle_rbf(n_steps):
    w = wl.permalloy_particle(n_steps=n_steps)
    lay = wl.rbf_layout((0, 0, 64), n_side=20, holes=0, seed=5)
    lay["s"] = lay["s"] + np.random.default_rng(6).uniform(-1.0, 1.0, lay["s"].size)
    return w, lay


def oracle_design_gradient(w, lay, n_steps):
    """dJ/ds by the oracle chain: RBF map -> phi -> (forward, adjoint) -> dJ/dphi -> VJP."""
    D2 = w.design[0]
    ctr = (lay["xc"], lay["yc"])
    phi, dphi, sc = orbf.pnorm_levelset(lay["s"], ctr, lay["c"], lay["p"], D2)
    w.phi = phi
    r = oracle_gradient(w, n_steps=n_steps)
    ds = orbf.pnorm_levelset_vjp(lay["s"], ctr, lay["c"], lay["p"], D2, r["dphi"].reshape(D2.shape), dphi, sc)
    return r["J"], ds


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_design_gradient_and_adam_steps_match_oracle(dtype):
    """The paper's loop on the permalloy particle (20x20 RBFs over the whole
    64x64 mesh, 16 RK4 steps): s -> phi -> psi -> J and dJ/ds through the
    autograd functions, then an Adam step, three times.  At every step J and
    dJ/ds are checked against the oracle chain at the current s, and the Adam
    update against the oracle's Adam fed the same gradient and moments."""
    import torch
    from paper_2411_19109_amd import llg
    from paper_2411_19109_amd.autograd import LevelSetLLG, RBFLevelSetFn
    from _helpers import gpu_objective
    n = 16
    w, lay = particle_rbf(n)
    rbfm = gpu_map(lay, w.design[0], dtype)
    solver = llg.Solver(w.problem, dtype=dtype, max_steps=n, design=w.design)
    obj = gpu_objective(w)
    s = s_dev(lay["s"]).requires_grad_()
    opt = llg.Adam(s.numel(), lr=0.05)
    m_o = v_o = np.zeros(s.numel())
    for t in range(1, 4):
        s.grad = None
        phi = RBFLevelSetFn.apply(s, rbfm)
        J = LevelSetLLG.apply(phi, to_dev(w.m0, dtype), solver, obj, n, w.heaviside_a,
                              to_dev(w.psi_fixed, dtype), True)
        J.backward()
        torch.cuda.synchronize()
        s_now, g_now = to_np(s.detach()), to_np(s.grad)
        Jo, dso = oracle_design_gradient(w, dict(lay, s=s_now), n)
        say("design step", t, dtype, "J gpu/oracle", float(J.item()), Jo, "dJ/ds rel L2", rel_l2(g_now, dso))
        assert abs(float(J.item()) - Jo) <= (1e-10 if dtype == "f64" else 1e-4) * abs(Jo)
        assert rel_l2(g_now, dso) <= (1e-8 if dtype == "f64" else 1e-3)
        opt.step(s.data, s.grad)
        s_o, m_o, v_o = orbf.adam_step(s_now, g_now, m_o, v_o, t, lr=0.05)
        torch.cuda.synchronize()
        assert rel_max(to_np(s.detach()), s_o) <= 1e-13
        assert np.abs(s_o - s_now).max() > 0.04
    solver.close()
