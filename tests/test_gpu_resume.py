"""A run split at step K and resumed from its state at t0 = K dt ends where the
unsplit run ends.  The step map depends on the time only through the drive,
so an undriven FP64 run resumes bit for bit; a driven one differs by the
rounding of the stage times (t0 + k dt against (K + k) dt) in the drive's
argument; an FP32 run differs by the state's low part, which the compensated
update keeps inside one run and a split drops (one rounding of m per node)."""
import numpy as np
import pytest

from _helpers import gpu_solver, oracle_psi, say, to_dev, to_np
from paper_2411_19109_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _split(w, dtype, n, k):
    import torch
    s = gpu_solver(w, dtype, max_steps=n)
    psi = to_dev(oracle_psi(w), dtype)
    m0 = to_dev(w.m0, dtype)
    dt = w.problem.dt
    full, _ = s.forward(psi, m0, n)
    mid, _ = s.forward(psi, m0, k)
    end, _ = s.forward(psi, mid, n - k, t0=k * dt)
    torch.cuda.synchronize()
    out = to_np(full).astype(np.float64), to_np(end).astype(np.float64)
    s.close()
    return out


def test_undriven_fp64_resumes_bitwise():
    w = wl.permalloy_particle()
    say("particle 64x64 fp64, 60 steps split at 23")
    a, b = _split(w, "f64", 60, 23)
    assert np.abs(a - w.m0.reshape(-1)).max() > 1e-6  # the state has moved
    assert np.array_equal(a, b)


def test_driven_fp64_resumes_to_time_rounding():
    w = wl.yig_demux(n_steps=80, nx=64, ny=40, D=20, wg=8)
    say("driven demux 64x40 fp64, 80 steps split at 37")
    a, b = _split(w, "f64", 80, 37)
    assert np.abs(a - w.m0.reshape(-1)).max() > 1e-9
    assert np.abs(a - b).max() <= 1e-13


def test_fp32_resumes_to_one_rounding():
    w = wl.permalloy_particle()
    say("particle 64x64 fp32, 60 steps split at 23")
    a, b = _split(w, "f32", 60, 23)
    d = np.abs(a - b).max()
    say("max |m_split - m_full|", d)
    assert d <= 1e-6
