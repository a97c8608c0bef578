"""The allocation-free entry point llg_shape_penalty_noalloc against
llg_shape_penalty (the same kernels, with the handle's own scratch): two calls
in a row on one GPU, the second on a smaller grid, each bit for bit equal to
the allocating call on the same input; FP64 and FP32; with and without the
gradient."""
import numpy as np
import pytest

from _helpers import say

pytestmark = pytest.mark.gpu


def _handle(nx, ny, nz, dtype):
    from paper_2411_19109_amd import llg, workloads as wl
    p = wl.Problem(nx=nx, ny=ny, nz=nz, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5, A=1.3e-11, terms=wl.TERM_EXCH, dt=1e-13)
    return llg.Solver(p, dtype=dtype, max_steps=1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_shape_penalty_matches_the_allocating_call(dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(11)
    args = (0.7, 310.0, 0.05, 80.0, 61.0)  # xi, S_target, nu, x0, y0
    for (nx, ny, nz) in ((197, 153, 2), (41, 29, 1)):  # the second call on a smaller grid
        say("noalloc shape penalty", dtype, (nx, ny, nz))
        s = _handle(nx, ny, nz, dtype)
        psi = torch.as_tensor(rng.uniform(0.0, 1.0, nx * ny * nz), dtype=td, device="cuda:0")
        J = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
        g = torch.full((s.N,), np.nan, dtype=torch.float64, device="cuda:0")
        s.shape_penalty_noalloc(psi, *args, J, g)
        J2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
        s.shape_penalty_noalloc(psi, *args, J2, None)
        Jr, gr = s.shape_penalty(psi, *args)
        torch.cuda.synchronize()
        assert np.isfinite(Jr.item()) and Jr.item() > 0
        assert J.item() == Jr.item() and J2.item() == Jr.item()
        assert np.array_equal(g.cpu().numpy(), gr.cpu().numpy())
        s.close()
