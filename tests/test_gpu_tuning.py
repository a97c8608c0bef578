"""Launch configurations and the autotuner: for a given FFT radix every valid
tiling of the column and row kernels gives the same bits (the passes of a
signal and the per-node arithmetic do not depend on the tiling); another radix
changes only the rounding order of the transforms; invalid configurations are
rejected on the host; the autotuner picks a valid one."""
import numpy as np
import pytest

from _helpers import gpu_gradient, gpu_solver, say
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _same(g, ref):
    assert g["J"] == ref["J"]
    for k in ("dpsi", "dm0", "mT"):
        assert np.array_equal(g[k], ref[k]), k


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_launch_configs_bitwise(dtype):
    from paper_2411_19109_amd import llg
    from test_gpu_parity import tiny_workload
    w = tiny_workload(21, 13, 1, kind=wl.OBJ_PORT_MY2, n_steps=12)
    s = gpu_solver(w, dtype, max_steps=12)
    base = s.launch_config()
    say("default launch config", base, dtype)
    cr, fr, br = base[2], base[4], base[6]
    ref = gpu_gradient(w, dtype, solver=s)
    tried = 0
    for tk in (1, 2, 4, 8, 16):
        for ct in (64, 128, 256):
            for ft, bt, nv in ((64, 128, 4), (128, 64, 7), (256, 256, 4), (192, 320, 7)):
                cfg = (tk, ct, cr, ft, fr, bt, br, nv)
                try:
                    s.set_launch_config(*cfg)
                except llg.LLGError:
                    continue
                assert s.launch_config() == cfg
                _same(gpu_gradient(w, dtype, solver=s), ref)
                tried += 1
    assert tried >= 10
    # other radices: the same values up to the rounding of the transforms
    tol = 1e-12 if dtype == "f64" else 2e-5
    for rc, rf, rb in ((4, 4, 4), (8, 4, 8), (4, 8, 4)):
        s.set_launch_config(1, 256, rc, 256, rf, 256, rb, 4)
        g = gpu_gradient(w, dtype, solver=s)
        assert abs(g["J"] - ref["J"]) <= tol * abs(ref["J"])
        assert np.abs(g["mT"] - ref["mT"]).max() <= tol
        assert np.linalg.norm(g["dpsi"] - ref["dpsi"]) <= 50 * tol * np.linalg.norm(ref["dpsi"])
    bad = [(3, 128, cr, 128, fr, 128, br, 4), (1, 100, cr, 128, fr, 128, br, 4), (1, 128, cr, 1024, fr, 128, br, 4),
           (1, 128, cr, 128, fr, 128, br, 5), (1, 128, 2, 128, fr, 128, br, 4)]
    if dtype == "f64":
        bad.append((1, 256, 16, 256, 8, 256, 8, 4))
    for cfg in bad:
        with pytest.raises(llg.LLGError):
            s.set_launch_config(*cfg)
    s.close()


def test_autotune_keeps_results():
    from paper_2411_19109_amd import llg
    from test_gpu_batch import antenna_ports, ragged_set, run_batch
    n = 10
    ws = antenna_ports(ragged_set(n))
    say("autotune on a ragged batch")
    ref = run_batch(ws, "f32", n)
    b = llg.Batch([w.problem for w in ws], dtype="f32", max_steps=n,
                  masks=[dict(antenna=w.antenna, port1=w.port1, port2=w.port2, design=w.design) for w in ws])
    cfg = b.autotune()
    say("autotuned", cfg)
    assert cfg[0] in (1, 2, 4, 8, 16) and cfg[1] % 64 == 0 and cfg[3] % 64 == 0 and cfg[5] % 64 == 0
    assert cfg[2] in (4, 8, 16) and cfg[4] in (4, 8, 16) and cfg[6] in (4, 8, 16) and cfg[7] in (4, 7)
    b.close()
    out = run_batch(ws, "f32", n, tune=True)
    for i in range(len(ws)):
        # the tuned radices may round the transforms differently: FP32 tolerance
        assert abs(out[i]["J"] - ref[i]["J"]) <= 1e-4 * abs(ref[i]["J"])
        assert np.abs(out[i]["mT"] - ref[i]["mT"]).max() <= 1e-5
        assert np.linalg.norm(out[i]["dpsi"] - ref[i]["dpsi"]) <= 1e-3 * np.linalg.norm(ref[i]["dpsi"])


def test_row_staging_choice_is_bitwise_neutral():
    """A 512-wide grid where the forward row kernel stages its neighbour rows in
    LDS at 512 threads (LDS and registers then allow two blocks per CU either
    way) but reads them from memory at 192 threads (four blocks instead of
    two): both give the same bits."""
    from test_gpu_parity import tiny_workload
    w = tiny_workload(512, 3, 1, kind=wl.OBJ_PORT_MY2, n_steps=6)
    s = gpu_solver(w, "f32", max_steps=6)
    base = s.launch_config()
    outs = []
    for ft in (512, 192):
        s.set_launch_config(base[0], base[1], base[2], ft, 16, base[5], base[6], base[7])
        say("launch", s.launch_config())
        outs.append(gpu_gradient(w, "f32", solver=s))
    # the trajectory and the gradient are bitwise equal; J itself is a float64
    # sum over each row pair's port nodes whose order follows the row block
    # size (one node per thread at 512 threads, up to three at 192), so it may
    # differ in its last bits
    for k in ("dpsi", "dm0", "mT"):
        assert np.array_equal(outs[1][k], outs[0][k]), k
    assert abs(outs[1]["J"] - outs[0]["J"]) <= 4e-16 * abs(outs[0]["J"])
    s.close()
