"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/llg.h declares, and rejects invalid arguments on the
host before any device work."""
import ctypes
import math
import os
import re

import pytest

from paper_2411_19109_amd import llg
from paper_2411_19109_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "llg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s+(llg_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_documented_boundary():
    names = declared_functions()
    for need in ["llg_create", "llg_destroy", "llg_levelset_to_Ms", "llg_levelset_to_Ms_vjp", "llg_forward",
                 "llg_objective", "llg_adjoint", "llg_field", "llg_query_memory", "llg_last_error"]:
        assert need in names
    assert set(names) == set(llg.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = llg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.llg_version().decode().startswith("llg-mi355x")


def _bad(**kw):
    p = wl.yig_waveguide_plain().problem
    pc = llg.make_problem(p, "f32", 10)
    for k, v in kw.items():
        setattr(pc, k, v)
    h = ctypes.c_void_p()
    rc = llg.lib().llg_create(ctypes.byref(pc), None, ctypes.byref(h))
    return rc, llg.lib().llg_last_error().decode(), h


@pytest.mark.parametrize("field,value", [("nx", 0), ("dt", 0.0), ("dt", float("nan")), ("Ms", -1.0),
                                         ("dtype", 7), ("terms", 64), ("max_steps", 0), ("ckpt_policy", 9),
                                         ("nz", 9), ("alpha0", -0.1), ("dx", 0.0)])
def test_create_rejects_invalid_problem_on_host(field, value):
    rc, msg, h = _bad(**{field: value})
    assert rc in (llg.LLG_EINVAL, llg.LLG_ESHAPE)
    assert msg
    assert not h.value


def test_null_arguments_are_rejected():
    L = llg.lib()
    assert L.llg_create(None, None, None) == llg.LLG_EINVAL
    assert L.llg_forward(None, None, None, 0.0, 1, None, None, None, None) == llg.LLG_EINVAL
    assert L.llg_adjoint(None, None, None, None, None, None, None, None) == llg.LLG_EINVAL
    assert L.llg_destroy(None) == llg.LLG_OK
    assert "NULL" in L.llg_last_error().decode()


def test_query_memory_matches_checkpoint_layout():
    p = wl.permalloy_particle().problem
    n = 2000
    K = math.ceil(math.sqrt(n))
    nsnap = math.ceil(n / K)
    N3 = 3 * p.n
    # a float snapshot holds the state's high and low parts (2 * N3 floats), a double one N3 doubles;
    # several segments: the stage store is double-buffered (recompute / transpose overlap)
    assert llg.query_memory(p, n, llg.LLG_CKPT_SQRT) == (2 * nsnap * N3 + 2 * 8 * K * N3) * 4
    assert llg.query_memory(p, n, llg.LLG_CKPT_ALL) == (2 * N3 + 8 * n * N3) * 4
    assert llg.query_memory(p, n, llg.LLG_CKPT_SQRT, dtype="f64") == (nsnap * N3 + 2 * 8 * K * N3) * 8
    assert llg.query_memory(p, n, llg.LLG_CKPT_SQRT, ckpt_param=n) == (2 * N3 + 8 * n * N3) * 4
    # sqrt(n) growth: 100x more steps costs ~10x the store
    r = llg.query_memory(p, 200000, llg.LLG_CKPT_SQRT) / llg.query_memory(p, 2000, llg.LLG_CKPT_SQRT)
    assert 8 < r < 12
    # binomial: s snapshots + one step's stage states, independent of n
    for steps in (64, 2000, 50000):
        assert llg.query_memory(p, steps, llg.LLG_CKPT_BINOMIAL, 32) == (2 * 32 * N3 + 8 * N3) * 4
    assert llg.query_memory(p, 10, llg.LLG_CKPT_BINOMIAL, 32) == (2 * 10 * N3 + 8 * N3) * 4
    assert llg.query_memory(p, 10, llg.LLG_CKPT_BINOMIAL, 32, dtype="f64") == (10 * N3 + 8 * N3) * 8


def test_memory_report_large_3d_device():
    """Checkpoint store of the 512x256x4 FP32 device over 50 000 steps: keeping
    every stage state would need 8 * 50 000 * 3N * 4 B (> 288 GB of HBM); the sqrt
    and binomial schedules need a few GB and a fraction of a GB."""
    p = wl.yig_device_3d().problem
    n = 50000
    N3 = 3 * p.n
    full = llg.query_memory(p, n, llg.LLG_CKPT_ALL)
    sq = llg.query_memory(p, n, llg.LLG_CKPT_SQRT)
    bi = llg.query_memory(p, n, llg.LLG_CKPT_BINOMIAL, 32)
    assert full == (2 * N3 + 8 * n * N3) * 4 and full > 288e9
    assert sq < 26e9 and bi < 0.5e9
    assert bi == (2 * 32 + 8) * N3 * 4


def _optimal_reversal_steps(l, s):
    """Fewest forward steps that reverse l steps when the state at the start is
    kept and s further snapshots are free (dynamic programming over the split)."""
    import functools

    @functools.lru_cache(None)
    def c(l, s):
        if l == 1:
            return 1
        best = l * (l + 1) // 2  # every step reached again from the start
        if s > 0:
            for d in range(1, l):
                best = min(best, d + c(l - d, s - 1) + c(d, s))
        return best
    return c(l, s)


def test_binomial_schedule_recomputation():
    from math import comb
    assert llg.query_recompute(2000, llg.LLG_CKPT_SQRT) == 2000
    assert llg.query_recompute(2000, llg.LLG_CKPT_ALL) == 2000
    for n in range(1, 70):
        for slots in range(1, 8):
            rec = llg.query_recompute(n, llg.LLG_CKPT_BINOMIAL, slots)
            r = next(r for r in range(n + 1) if comb(slots + r, slots) >= n)
            assert n <= rec <= (r + 1) * n
            # the forward pass places the first snapshots, so the adjoint never
            # recomputes more than an optimal reversal that starts from m_0 alone
            assert rec <= _optimal_reversal_steps(n, slots - 1)
        assert llg.query_recompute(n, llg.LLG_CKPT_BINOMIAL, 1) == n * (n + 1) // 2
        assert llg.query_recompute(n, llg.LLG_CKPT_BINOMIAL, n) == n
    # the 50 000-step device with 32 snapshots: r = 4 since C(36, 4) >= 50 000
    assert llg.query_recompute(50000, llg.LLG_CKPT_BINOMIAL, 32) <= 4 * 50000


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(llg, "_lib", None)
    monkeypatch.setattr(llg, "LIB_PATH", os.path.join(ROOT, "no_such_libllg.so"))
    with pytest.raises(RuntimeError, match="not built"):
        llg.lib()


def test_rbf_work_len_and_host_side_rejections():
    L = llg.lib()
    v = ctypes.c_int64(0)
    assert L.llg_rbf_work_len(64, 64, 400, ctypes.byref(v)) == llg.LLG_OK
    assert v.value > 2 + 400
    assert L.llg_rbf_work_len(0, 64, 400, ctypes.byref(v)) == llg.LLG_ESHAPE
    assert L.llg_rbf_work_len(64, 64, 0, ctypes.byref(v)) == llg.LLG_EINVAL
    assert L.llg_rbf_work_len(64, 64, 400, None) == llg.LLG_EINVAL
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its host checks first
    args = dict(dtype=llg.LLG_F32, nx=8, ny=8, n=4, c=1.0, p=90.0)

    def call(**kw):
        a = dict(args, **kw)
        return L.llg_rbf_levelset(a["dtype"], a["nx"], a["ny"], a["n"], fake, fake, a["c"], a["p"], fake, 1,
                                  kw.get("phi", fake), None, fake, None)
    assert call(dtype=5) == llg.LLG_EINVAL
    assert call(p=0.5) == llg.LLG_EINVAL
    assert call(p=float("nan")) == llg.LLG_EINVAL
    assert call(c=float("inf")) == llg.LLG_EINVAL
    assert call(nx=-1) == llg.LLG_ESHAPE
    assert call(phi=None) == llg.LLG_EINVAL
    assert "NULL" in L.llg_last_error().decode()
    assert L.llg_rbf_levelset_vjp(llg.LLG_F64, 8, 8, 4, fake, fake, 1.0, 90.0, fake, fake, None, fake, fake,
                                  None) == llg.LLG_EINVAL
    assert L.llg_adam_step(4, fake, fake, fake, fake, 0, 1e-2, 0.9, 0.999, 1e-8, None) == llg.LLG_EINVAL
    assert L.llg_adam_step(4, fake, fake, fake, fake, 1, 1e-2, 1.0, 0.999, 1e-8, None) == llg.LLG_EINVAL
    assert L.llg_adam_step(4, None, fake, fake, fake, 1, 1e-2, 0.9, 0.999, 1e-8, None) == llg.LLG_EINVAL


def test_shape_penalty_rejects_null_handle():
    L = llg.lib()
    assert L.llg_shape_penalty(None, None, 0.05, 30.0, 1.0, 0.0, 0.0, None, None, None) == llg.LLG_EINVAL


def test_adaptive_entries_reject_null_handle():
    """The stage-store switch and both adaptive adjoints check their handle
    before touching the device."""
    L = llg.lib()
    assert L.llg_set_keep_stages(None, 1) == llg.LLG_EINVAL
    assert "NULL" in L.llg_last_error().decode()
    assert L.llg_adjoint_adaptive(None, None, None, None, None, None, None) == llg.LLG_EINVAL
    assert L.llg_adjoint_continuous(None, None, None, None, 2, None, None, None) == llg.LLG_EINVAL
