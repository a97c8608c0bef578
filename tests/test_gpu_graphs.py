"""HIP-graph replay of the forward / adjoint launch sequences: every replay,
with eager work and synchronisations in between, gives the bits of the eager
(graph-free) run, for the overlapped sqrt schedule, the binomial schedule, both
objectives and a ragged batch."""
import numpy as np
import pytest

from _helpers import gpu_gradient, gpu_solver, say, to_dev, to_np
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _eager_work():
    import torch
    x = torch.arange(1 << 16, device="cuda:0", dtype=torch.float32)
    y = (x * 2.0).sum()
    torch.cuda.synchronize()
    return float(y.item())


def _same(g, ref):
    assert g["J"] == ref["J"]
    for k in ("dpsi", "dm0", "dphi", "mT"):
        assert np.array_equal(g[k], ref[k]), k


@pytest.mark.parametrize("kind,policy,param", [(wl.OBJ_PORT_MY2, 0, 5), (wl.OBJ_ENERGY_AREA, 0, 0),
                                               (wl.OBJ_PORT_MY2, 2, 3)])
def test_graph_replays_match_eager(kind, policy, param):
    from test_gpu_parity import tiny_workload
    w = tiny_workload(13, 9, 1, kind=kind, n_steps=30)
    say("graphs: objective", kind, "policy", policy, "param", param)
    ref = gpu_gradient(w, "f32", ckpt_policy=policy, ckpt_param=param)
    ref["solver"].close()
    s = gpu_solver(w, "f32", max_steps=30, ckpt_policy=policy, ckpt_param=param)
    s.set_graphs(True)
    for rep in range(3):
        g = gpu_gradient(w, "f32", solver=s)
        _same(g, ref)
        _eager_work()
    # another signature (shorter run) captures new graphs and still matches eager
    ref2 = gpu_gradient(w, "f32", n_steps=17, ckpt_policy=policy, ckpt_param=param)
    ref2["solver"].close()
    for rep in range(2):
        _same(gpu_gradient(w, "f32", n_steps=17, solver=s), ref2)
        _same(gpu_gradient(w, "f32", solver=s), ref)
    s.set_graphs(False)
    _same(gpu_gradient(w, "f32", solver=s), ref)
    s.close()


def test_batch_graph_replays_match_eager():
    import torch
    from paper_2411_19109_amd import llg
    from test_gpu_batch import ragged_set
    n = 20
    ws = ragged_set(n)
    say("batch graphs")

    def run(b):
        phis = [to_dev(w.phi, "f32") for w in ws]
        psis = b.levelset_to_psi(phis, ws[0].heaviside_a, [to_dev(w.psi_fixed, "f32") for w in ws])
        obj = llg.make_objective(wl.OBJ_PORT_MY2, n_start=ws[0].obj_n_start)
        mT, J = b.forward(psis, [to_dev(w.m0, "f32") for w in ws], n, obj=obj)
        g, dm0 = b.adjoint(psis, obj, want_dm0=True)
        torch.cuda.synchronize()
        return [dict(J=float(J[i].item()), mT=to_np(mT[i]), dpsi=to_np(g[i]), dm0=to_np(dm0[i])) for i in range(len(ws))]

    def make():
        return llg.Batch([w.problem for w in ws], dtype="f32", max_steps=n, ckpt_param=4,
                         masks=[dict(antenna=w.antenna, port1=w.port1, port2=w.port2, design=w.design) for w in ws])
    b = make()
    ref = run(b)
    b.close()
    b = make()
    b.set_graphs(True)
    for rep in range(3):
        out = run(b)
        for i in range(len(ws)):
            assert out[i]["J"] == ref[i]["J"]
            for k in ("mT", "dpsi", "dm0"):
                assert np.array_equal(out[i][k], ref[i][k]), (rep, i, k)
        _eager_work()
    b.close()


def test_long_calls_run_without_graphs():
    """Calls of more than 2 000 RK4 steps run their launches directly even with
    graphs enabled (longer sequences are not captured): same bits as with graphs
    off, and a 2 000-step call on the same handle still replays."""
    from test_gpu_parity import tiny_workload
    w = tiny_workload(7, 5, 1, kind=wl.OBJ_ENERGY_AREA, n_steps=2001)
    say("graphs enabled, 2001- and 2000-step calls")
    ref = gpu_gradient(w, "f32", n_steps=2001)
    ref["solver"].close()
    ref2 = gpu_gradient(w, "f32", n_steps=2000)
    ref2["solver"].close()
    s = gpu_solver(w, "f32", max_steps=2001)
    s.set_graphs(True)
    for rep in range(2):
        _same(gpu_gradient(w, "f32", n_steps=2001, solver=s), ref)
        _same(gpu_gradient(w, "f32", n_steps=2000, solver=s), ref2)
        _eager_work()
    s.close()
