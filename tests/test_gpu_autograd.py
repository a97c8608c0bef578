"""The torch.autograd functions over the C ABI: the level-set + forward +
objective chain differentiated by J.backward() gives the same bits as the
explicit call sequence, matches the oracle's gradient, scales with the
incoming gradient, and a gradient of <w, m_T> through IntegrateLLG matches
central differences of the FP64 path; the batched function gives every
instance the gradient of the explicit batch call sequence, scaled per instance;
a backward after another forward on the handle is refused."""
import numpy as np
import pytest

from _helpers import gpu_gradient, gpu_objective, gpu_solver, oracle_gradient, rel_l2, say, to_dev, to_np
from paper_2411_19109_amd import workloads as wl
from test_gpu_parity import tiny_workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_levelset_llg_equals_call_sequence(dtype):
    import torch
    from paper_2411_19109_amd.autograd import LevelSetLLG
    w = tiny_workload(13, 9, 1, kind=wl.OBJ_ENERGY_AREA, n_steps=12)
    say("autograd energy objective", dtype)
    ref = gpu_gradient(w, dtype)
    s = ref["solver"]
    phi = to_dev(w.phi, dtype).requires_grad_()
    m0 = to_dev(w.m0, dtype).requires_grad_()
    J = LevelSetLLG.apply(phi, m0, s, gpu_objective(w), w.n_steps, w.heaviside_a, to_dev(w.psi_fixed, dtype), True)
    J.backward()
    torch.cuda.synchronize()
    say("J", float(J), ref["J"])
    assert float(J) == ref["J"]
    # the library's dJ/dphi is float64; the gradient takes phi's dtype
    npdt = np.float64 if dtype == "f64" else np.float32
    assert np.array_equal(to_np(phi.grad), ref["dphi"].astype(npdt).astype(np.float64))
    assert np.array_equal(to_np(m0.grad), ref["dm0"])
    s.close()


def test_composed_functions_match_oracle_and_scale():
    import torch
    from paper_2411_19109_amd.autograd import LevelSet, LLGObjective
    w = tiny_workload(16, 8, 1, kind=wl.OBJ_PORT_MY2, n_steps=12)
    say("autograd port objective, LevelSet -> LLGObjective, f64")
    s = gpu_solver(w, "f64", max_steps=w.n_steps)
    obj = gpu_objective(w)
    pf = to_dev(w.psi_fixed, "f64")
    grads = []
    for scale in (1.0, -2.5):
        phi = to_dev(w.phi, "f64").requires_grad_()
        m0 = to_dev(w.m0, "f64").requires_grad_()
        psi = LevelSet.apply(phi, s, w.heaviside_a, pf, True)
        J = LLGObjective.apply(psi, m0, s, obj, w.n_steps)
        (scale * J).backward()
        torch.cuda.synchronize()
        grads.append((float(J), to_np(phi.grad), to_np(m0.grad)))
    r = oracle_gradient(w)
    J1, gphi, gm0 = grads[0]
    say("J gpu / oracle", J1, r["J"], "rel L2 dphi", rel_l2(gphi, r["dphi"]))
    assert abs(J1 - r["J"]) <= 1e-10 * abs(r["J"])
    assert rel_l2(gphi, r["dphi"]) <= 1e-9
    assert rel_l2(gm0, r["dm0"]) <= 1e-9
    assert grads[1][0] == J1
    assert np.allclose(grads[1][1], -2.5 * gphi, rtol=1e-14, atol=0)
    assert np.allclose(grads[1][2], -2.5 * gm0, rtol=1e-14, atol=0)
    s.close()


def test_integrate_gradient_vs_central_differences():
    import torch
    from paper_2411_19109_amd.autograd import IntegrateLLG
    w = tiny_workload(9, 7, 1, kind=wl.OBJ_NONE, n_steps=10)
    say("autograd IntegrateLLG, <w, m_T>, f64, central differences")
    s = gpu_solver(w, "f64", max_steps=w.n_steps)
    rng = np.random.default_rng(11)
    N = w.problem.n
    psi0 = np.clip(np.asarray(w.psi_fixed, np.float64).reshape(-1) + 0.2, 0.05, 1.0)
    wt = to_dev(rng.standard_normal(3 * N), "f64")
    psi = to_dev(psi0, "f64").requires_grad_()
    m0 = to_dev(w.m0, "f64").requires_grad_()
    L = (wt * IntegrateLLG.apply(psi, m0, s, w.n_steps)).sum()
    L.backward()
    torch.cuda.synchronize()
    g_psi, g_m0 = to_np(psi.grad), to_np(m0.grad)

    def loss(p, m):
        mT = IntegrateLLG.apply(to_dev(p, "f64"), to_dev(m, "f64"), s, w.n_steps)
        return float((wt * mT).sum())

    vp = rng.standard_normal(N)
    vm = rng.standard_normal(3 * N)
    m0n = np.asarray(w.m0, np.float64).reshape(-1)
    h = 1e-6
    fd_p = (loss(psi0 + h * vp, m0n) - loss(psi0 - h * vp, m0n)) / (2 * h)
    fd_m = (loss(psi0, m0n + h * vm) - loss(psi0, m0n - h * vm)) / (2 * h)
    say("psi: adjoint", g_psi @ vp, "fd", fd_p, " m0: adjoint", g_m0 @ vm, "fd", fd_m)
    assert abs(g_psi @ vp - fd_p) <= 1e-7 * max(1.0, abs(fd_p))
    assert abs(g_m0 @ vm - fd_m) <= 1e-7 * max(1.0, abs(fd_m))
    s.close()


def test_backward_after_another_forward_is_refused():
    import torch
    from paper_2411_19109_amd import llg
    from paper_2411_19109_amd.autograd import LLGObjective
    w = tiny_workload(7, 5, 1, kind=wl.OBJ_PORT_MY2, n_steps=6)
    s = gpu_solver(w, "f64", max_steps=w.n_steps)
    psi = to_dev(np.full(w.problem.n, 0.8), "f64").requires_grad_()
    m0 = to_dev(w.m0, "f64")
    J = LLGObjective.apply(psi, m0, s, gpu_objective(w), w.n_steps)
    s.forward(psi.detach(), m0, w.n_steps)  # the handle now records another trajectory
    with pytest.raises(llg.LLGError):
        J.backward()
    torch.cuda.synchronize()
    s.close()


def test_batch_levelset_llg_equals_batch_call_sequence():
    import torch
    from paper_2411_19109_amd import llg
    from paper_2411_19109_amd.autograd import BatchLevelSetLLG
    from test_gpu_batch import antenna_ports, ragged_set, run_batch
    n = 10
    ws = antenna_ports(ragged_set(n))
    say("autograd batch of", len(ws), "ragged instances, f32")
    ref = run_batch(ws, "f32", n)
    b = llg.Batch([w.problem for w in ws], dtype="f32", max_steps=n,
                  masks=[dict(antenna=w.antenna, port1=w.port1, port2=w.port2, design=w.design) for w in ws])
    obj = llg.make_objective(wl.OBJ_PORT_MY2, n_start=ws[0].obj_n_start)
    phis = [to_dev(w.phi, "f32").requires_grad_() for w in ws]
    Js = BatchLevelSetLLG.apply(b, obj, n, ws[0].heaviside_a, [to_dev(w.psi_fixed, "f32") for w in ws], True,
                                [to_dev(w.m0, "f32") for w in ws], *phis)
    wts = torch.tensor([1.0, -0.5, 2.0, 0.25][:len(ws)], dtype=torch.float64, device=Js.device)
    (wts * Js).sum().backward()
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        assert float(Js[i]) == ref[i]["J"]
        # the explicit sequence's float64 dJ/dphi, scaled and rounded to phi's dtype
        want = (float(wts[i]) * ref[i]["dphi"]).astype(np.float32).astype(np.float64)
        assert np.array_equal(to_np(phis[i].grad), want), i
    b.close()


def test_readme_usage():
    """The usage shown in the README: autotuned FP32 solver on the particle
    workload, J.backward() through LevelSetLLG, against the oracle gradient of
    the same map (FP32 tolerance)."""
    import torch
    from paper_2411_19109_amd import llg
    from paper_2411_19109_amd.autograd import LevelSetLLG
    from _helpers import oracle_gradient
    w = wl.permalloy_particle(n_steps=200)  # a prefix keeps the oracle quick; the calls are the README's
    s = llg.Solver(w.problem, dtype="f32", max_steps=w.n_steps, design=w.design)
    s.autotune()
    obj = llg.make_objective(w.objective, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area)
    dev = torch.device("cuda:0")
    phi = torch.as_tensor(w.phi.reshape(-1), dtype=torch.float32, device=dev).requires_grad_()
    m0 = torch.as_tensor(w.m0.reshape(-1), dtype=torch.float32, device=dev)
    psi_fixed = torch.as_tensor(w.psi_fixed.reshape(-1), dtype=torch.float32, device=dev)
    J = LevelSetLLG.apply(phi, m0, s, obj, w.n_steps, w.heaviside_a, psi_fixed, True)
    J.backward()
    torch.cuda.synchronize()
    r = oracle_gradient(w)
    say("README usage: J", float(J), r["J"], "rel L2 dphi", rel_l2(to_np(phi.grad), r["dphi"]))
    assert abs(float(J) - r["J"]) <= 1e-4 * abs(r["J"])
    assert rel_l2(to_np(phi.grad), r["dphi"]) <= 1e-3
    s.close()
