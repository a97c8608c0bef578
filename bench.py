"""Throughput of the level-set LLG gradient path on one MI355X.

One "step" is one full gradient evaluation of the workload: level set -> psi,
n RK4 steps of the LLG equation with checkpoints, the objective, the
checkpointed discrete adjoint back to t0, and the chain rule to dJ/dphi.
Inputs are resident in device memory before the timed region starts.

The default workload is the batched sweep: 32 seeded demultiplexer designs x
2 drive frequencies = 64 instances on ragged grids (128..256 x 64..128 nodes,
1.15 M nodes in all), 10 000 RK4 steps each, FP32, one launch sequence for
the whole batch.  Beside it the same 64 instances are solved one after the
other as plain single-instance calls (the batched-over-plain ratio), and the
float64 oracle is timed on the host's cores.

  python bench.py [--steps K] [--warmup W]
                  [--workload sweep|particle|particle_curve|particle_adaptive|waveguide|demux|demux_spectral|
                              device3d|probe|rbf]

Prints ONE JSON line.  The metric is LLG cell-steps per second of the forward
+ adjoint run: nodes * RK4 steps / wall time of one gradient evaluation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LLG cell-steps/s fwd+adjoint; grad time/iter, batched vs plain at stated tol"
SWEEP_NAME = "yig_demux_sweep_64x_10000steps_grad"
HBM_PEAK_GBS = 8000.0


def make_workload(name):
    from paper_2411_19109_amd import workloads as wl
    if name == "particle":
        return wl.permalloy_particle()
    if name == "waveguide":
        w = wl.yig_waveguide_plain()
        w.objective = wl.OBJ_ENERGY_AREA
        return w
    if name == "demux":
        return wl.yig_demux()
    if name == "demux_spectral":
        return wl.yig_demux_two_tone()
    if name == "particle_curve":
        return wl.sw_particle_curve()
    if name == "device3d":
        return wl.yig_device_3d()
    raise SystemExit(f"unknown workload {name}")


class GradientStep:
    """Device-resident inputs and one gradient evaluation through the C ABI."""

    def __init__(self, w, graphs=True, tune=True, launch_file=None):
        import torch
        from paper_2411_19109_amd import llg, workloads as wl
        self.w = w
        self.td = torch.float64 if w.dtype == "f64" else torch.float32
        dev = torch.device("cuda:0")
        t0 = time.perf_counter()
        self.solver = llg.Solver(w.problem, dtype=w.dtype, max_steps=w.n_steps, antenna=w.antenna, port1=w.port1,
                                 port2=w.port2, design=w.design)
        torch.cuda.synchronize()
        self.t_create = time.perf_counter() - t0  # handle, Newell spectrum, device buffers
        self.solver.set_graphs(graphs)
        t0 = time.perf_counter()
        if launch_file and os.path.exists(launch_file):
            # a launch configuration fixed by an earlier run (profiling runs reuse it)
            self.solver.set_launch_config(*[int(v) for v in open(launch_file).read().split()])
            self.launch = self.solver.launch_config()
        else:
            self.launch = self.solver.autotune() if tune else self.solver.launch_config()
            if launch_file:
                with open(launch_file, "w") as fh:
                    fh.write(" ".join(str(v) for v in self.launch) + "\n")
        torch.cuda.synchronize()
        self.t_tune = time.perf_counter() - t0
        self.phi = torch.as_tensor(w.phi.reshape(-1), dtype=self.td, device=dev).contiguous()
        self.psi_fixed = torch.as_tensor(w.psi_fixed.reshape(-1), dtype=self.td, device=dev).contiguous()
        self.m0 = torch.as_tensor(w.m0.reshape(-1), dtype=self.td, device=dev).contiguous()
        self.obj = llg.make_objective(w.objective, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area,
                                      n_start=w.obj_n_start, freqs=w.extra.get("freqs"), coef=w.extra.get("coef"),
                                      target=w.extra.get("target"), weight=w.extra.get("weight"))
        self.energy = w.objective == wl.OBJ_ENERGY_AREA

    def __call__(self):
        s, w = self.solver, self.w
        psi = s.levelset_to_psi(self.phi, w.heaviside_a, self.psi_fixed, extrude_z=True)
        mT, Jp = s.forward(psi, self.m0, w.n_steps, obj=self.obj)
        if self.energy:
            J, dJdm, dJdpsi_e, _ = s.objective(self.obj, psi, mT)
        else:
            J, dJdm, dJdpsi_e = Jp, None, None
        dJdpsi = s.adjoint(psi, self.obj, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e)
        return J, s.levelset_vjp(self.phi, dJdpsi, w.heaviside_a, extrude_z=True)

    def forward_only(self):
        s, w = self.solver, self.w
        psi = s.levelset_to_psi(self.phi, w.heaviside_a, self.psi_fixed, extrude_z=True)
        return s.forward(psi, self.m0, w.n_steps, obj=self.obj)


class SweepStep:
    """The batched sweep: 32 seeded designs x 2 drive frequencies on ragged grids,
    one gradient evaluation of every instance with one launch sequence."""

    def __init__(self, n_steps, graphs=True, tune=True, launch_file=None):
        import torch
        from paper_2411_19109_amd import llg, workloads as wl
        self.ws = wl.yig_demux_sweep(n_steps=n_steps)
        for w in self.ws:
            w.obj_n_start = n_steps // 2
        self.n_steps = n_steps
        dev = torch.device("cuda:0")
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float32, device=dev)
        t0 = time.perf_counter()
        self.batch = llg.Batch([w.problem for w in self.ws], dtype="f32", max_steps=n_steps,
                               masks=[dict(antenna=w.antenna, port1=w.port1, port2=w.port2, design=w.design)
                                      for w in self.ws])
        torch.cuda.synchronize()
        self.t_create = time.perf_counter() - t0
        self.batch.set_graphs(graphs)
        t0 = time.perf_counter()
        if launch_file and os.path.exists(launch_file):
            self.batch.set_launch_config(*[int(v) for v in open(launch_file).read().split()])
            self.launch = self.batch.launch_config()
        else:
            self.launch = self.batch.autotune() if tune else self.batch.launch_config()
            if launch_file:
                with open(launch_file, "w") as fh:
                    fh.write(" ".join(str(v) for v in self.launch) + "\n")
        torch.cuda.synchronize()
        self.t_tune = time.perf_counter() - t0
        self.phi = [t(w.phi) for w in self.ws]
        self.psif = [t(w.psi_fixed) for w in self.ws]
        self.m0 = [t(w.m0) for w in self.ws]
        self.obj = llg.make_objective(wl.OBJ_PORT_MY2, n_start=n_steps // 2)
        self.nodes = sum(w.problem.n for w in self.ws)

    def forward(self):
        """Level set and forward run with checkpoints (enqueued); (psis, J)."""
        b = self.batch
        psis = b.levelset_to_psi(self.phi, self.ws[0].heaviside_a, self.psif)
        _, J = b.forward(psis, self.m0, self.n_steps, obj=self.obj, want_m=False)
        return psis, J

    def backward(self, psis):
        """Adjoint of the last forward run and the level-set VJP (enqueued); dJ/dphi."""
        g = self.batch.adjoint(psis, self.obj)
        return self.batch.levelset_vjp(self.phi, g, self.ws[0].heaviside_a)

    def __call__(self):
        psis, J = self.forward()
        return J, self.backward(psis)


def sweep_plain(n_steps, count, graphs=True, tune=True):
    """The same instances as single-instance solves, one after the other."""
    from paper_2411_19109_amd import workloads as wl
    ws = wl.yig_demux_sweep(n_steps=n_steps)
    steps = []
    for w in ws[:count]:
        w.obj_n_start = n_steps // 2
        steps.append(GradientStep(w, graphs, tune))
    return steps, sum(w.problem.n for w in ws[:count])


def _profile_supported(solver):
    """False while a profiler collects hardware counters (the library refuses
    event-timed dispatches then, LLG_ENOTSUP)."""
    from paper_2411_19109_amd import llg
    try:
        solver.profile(True)
    except llg.LLGError as e:
        if e.code == llg.LLG_ENOTSUP:
            print(f"[bench] kernel event timing off: {e}", file=sys.stderr, flush=True)
            return False
        raise
    solver.profile(False)
    return True


def _oracle_worker(idx, n_steps, n_designs_steps):
    """Child process: the float64 oracle's gradient (forward + adjoint, store-all)
    of sweep instance idx over its first n_steps RK4 steps; prints one JSON
    line {"cells": nodes * n_steps, "secs": wall seconds}."""
    from oracle import adjoint as oadj
    from oracle import levelset as ols
    from oracle import micromag as omm
    from paper_2411_19109_amd import workloads as wl
    w = wl.yig_demux_sweep(n_steps=n_designs_steps)[idx]
    sim = omm.Sim(w.problem, antenna=w.antenna)
    psi = ols.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    obj = oadj.Objective(w.objective, n_start=0, port1=w.port1, port2=w.port2)
    print("ready", flush=True)
    sys.stdin.readline()  # the parent starts every worker's timed work at once
    t0 = time.perf_counter()
    oadj.gradient(sim, w.m0, psi, n_steps, obj)
    dt = time.perf_counter() - t0
    print(json.dumps({"cells": w.problem.n * n_steps, "secs": dt, "nodes": w.problem.n}), flush=True)


def _host_workers():
    """Worker processes for the host baseline: the CPUs this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_sweep(n_run, budget_s=10.0):
    """The oracle as it stands, on the host's cores: each worker process (one
    thread each) runs the float64 oracle's gradient of one sweep instance over a
    prefix of its RK4 steps.  One worker alone gives the one-core rate, then
    one worker per core runs concurrently (instances 0..P-1) for the all-core
    rate (sum of cell-steps / wall time of the slowest).  Worker processes are
    plain children that never touch the GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")

    def spawn(idx, n):
        return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", str(idx), str(n),
                                 str(n_run)], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env,
                                 cwd=ROOT)

    def result(p):
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed ({p.returncode})")
        return json.loads(out.strip().splitlines()[-1])

    def go(procs):
        for p in procs:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker did not start")
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
    probe = spawn(0, 4)
    go([probe])
    per_step = result(probe)["secs"] / 4
    n = max(4, min(n_run, int(budget_s / max(per_step, 1e-3))))
    one = spawn(0, n)
    go([one])
    one = result(one)
    P = _host_workers()
    procs = [spawn(i, n) for i in range(P)]
    go_ready = [p.stdout.readline().strip() == "ready" for p in procs]  # inputs and oracle objects set up
    if not all(go_ready):
        raise RuntimeError("oracle worker did not start")
    t0 = time.perf_counter()
    for p in procs:
        p.stdin.write("go\n")
        p.stdin.flush()
    res = [result(p) for p in procs]
    wall = time.perf_counter() - t0
    cells = sum(r["cells"] for r in res)
    return dict(value=cells / wall, unit="cell-steps/s", cores=P, kind="oracle",
                one_core_value=one["cells"] / one["secs"],
                sample=f"float64 NumPy oracle, forward+adjoint of the first {n} of {n_run} RK4 steps of sweep "
                       f"instances 0..{P - 1} ({res[0]['nodes']}..{max(r['nodes'] for r in res)} nodes), one "
                       f"single-threaded process per core, {P} concurrently ({wall:.1f} s wall); one core alone: "
                       f"instance 0, {one['secs']:.1f} s")


def cpu_baseline(w, budget_s=15.0):
    """The oracle as it stands, timed on the host on a bounded prefix of the
    same workload (forward + adjoint over the first n steps)."""
    from oracle import adjoint as oadj
    from oracle import levelset as ols
    from oracle import micromag as omm
    from paper_2411_19109_amd import workloads as wl
    sim = omm.Sim(w.problem, antenna=w.antenna)
    psi = ols.levelset_to_psi(w.phi, w.heaviside_a, w.design, w.psi_fixed)
    def obj(n):
        tg, wt = w.extra.get("target"), w.extra.get("weight")
        return oadj.Objective(w.objective, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area,
                              n_start=0, port1=w.port1, port2=w.port2, freqs=w.extra.get("freqs"),
                              coef=w.extra.get("coef"), target=None if tg is None else tg[:n],
                              weight=None if wt is None else wt[:n])
    n = 10
    t0 = time.perf_counter()
    oadj.gradient(sim, w.m0, psi, n, obj(n))
    dt = time.perf_counter() - t0
    n = max(10, min(w.n_steps, int(n * budget_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    oadj.gradient(sim, w.m0, psi, n, obj(n))
    dt = time.perf_counter() - t0
    return dict(value=w.problem.n * n / dt, unit="cell-steps/s", cores=1, kind="oracle",
                sample=f"float64 NumPy oracle, forward+adjoint of the first {n} of {w.n_steps} RK4 steps "
                       f"({dt:.1f} s, one host thread)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work per host worker")
    ap.add_argument("--sweep-steps", type=int, default=10000, help="RK4 steps per instance of the sweep workload")
    ap.add_argument("--plain-steps", type=int, default=1000,
                    help="RK4 steps per instance of the plain (one instance per call) sweep; 0 skips it")
    ap.add_argument("--oracle-worker", nargs=3, type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--n-steps", type=int, default=0,
                    help="override the workload's RK4 step count (short profiling runs; not a bench line)")
    ap.add_argument("--graphs", type=int, default=0, help="1: replay forward/adjoint as captured HIP graphs")
    ap.add_argument("--plain-graphs", type=int, default=1,
                    help="sweep: 1 (default) replays the plain path's per-instance launches as HIP graphs, its fastest form")
    ap.add_argument("--autotune", type=int, default=1, help="1: pick launch tiles with the library's autotuner at setup")
    ap.add_argument("--launch-file", default=None,
                    help="read the launch configuration from this file if it exists, else write the chosen one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--rbf-paper-sizes", type=int, default=1,
                    help="rbf workload: 1 also times one update at the paper's grid sizes (0 for counter runs)")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="skip the per-kernel event timing pass (counter runs need only the dispatches)")
    args = ap.parse_args()
    if args.oracle_worker:
        return _oracle_worker(*args.oracle_worker)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_19109_amd import llg

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "probe":
        return run_probe(args)
    if args.workload == "rbf":
        return run_rbf(args)
    if args.workload == "particle_adaptive":
        return run_adaptive(args)
    w = make_workload(args.workload)
    if args.n_steps > 0 and args.workload == "particle_curve":
        from paper_2411_19109_amd import workloads as wl
        w = wl.sw_particle_curve(n_steps=args.n_steps)  # the ramp and the target follow the run length
    elif args.n_steps > 0:
        w.n_steps = args.n_steps
        w.obj_n_start = min(w.obj_n_start, args.n_steps // 2)
    step = GradientStep(w, bool(args.graphs), bool(args.autotune), args.launch_file)
    print(f"[bench] workload {w.name}: {w.problem.nx}x{w.problem.ny}x{w.problem.nz} nodes, {w.n_steps} steps, "
          f"{w.dtype}, launch {step.launch}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        J, g = step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    print(f"[bench] timed {args.steps} steps: {sec * 1e3:.2f} ms per gradient (median {np.median(per_step):.2f} ms)",
          file=sys.stderr, flush=True)

    # forward alone (level set + RK4 steps with checkpoints), for the forward throughput
    fwd_ms = []
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step.forward_only()
        e1.record()
        torch.cuda.synchronize()
        fwd_ms.append(e0.elapsed_time(e1))
    fwd_ms = min(fwd_ms)
    print(f"[bench] forward alone: {fwd_ms:.2f} ms", file=sys.stderr, flush=True)

    # per-kernel device time over one more gradient with event bracketing
    roofline = None
    if not args.no_kernel_events and _profile_supported(step.solver):
        s = step.solver
        s.profile(True)
        step()
        torch.cuda.synchronize()
        s.profile(False)
        kinds = {}
        for k, name in llg.KIND_NAMES.items():
            ms, n, b = s.profile_read(k)
            if n:
                kinds[name] = dict(ms=ms, launches=n, bytes=b, avg_us=1e3 * ms / n, gbs=b / (ms * 1e-3) / 1e9)
        dom = max(kinds, key=lambda k: kinds[k]["ms"])
        d = kinds[dom]
        roofline = dict(bound="hbm", achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(d["gbs"] / HBM_PEAK_GBS, 5), traffic=measured_traffic(w.name, dom, step.launch),
                        kernel=dom, avg_launch_us=round(d["avg_us"], 3),
                        bytes_per_launch=round(d["bytes"] / d["launches"]))
        for name, v in kinds.items():
            print(f"[bench] {name}: {v['launches']} launches, avg {v['avg_us']:.2f} us, "
                  f"{v['gbs']:.1f} GB/s algorithmic", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_budget)
        print(f"[bench] cpu baseline: {cpu['sample']}", file=sys.stderr, flush=True)

    N = w.problem.n
    out = {
        "metric": METRIC,
        "value": N * w.n_steps / sec,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": [w.problem.nx, w.problem.ny, w.problem.nz],
                   "rk4_steps": w.n_steps, "checkpoint": "sqrt", "grad_ms": round(sec * 1e3, 3),
                   "grad_ms_median": round(float(np.median(per_step)), 3),
                   "forward_ms": round(fwd_ms, 3), "forward_cell_steps_per_s": N * w.n_steps / (fwd_ms * 1e-3),
                   "hip_graphs": bool(args.graphs), "launch": list(step.launch),
                   "setup_s": {"create": round(step.t_create, 3), "launch_tuning": round(step.t_tune, 3)},
                   "objective_J": float(J.item())},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# the launch-configuration entries each kernel class's tiling depends on
# (column: x-bins per block, threads, radix; forward rows: threads, radix;
# backward rows: threads, radix, staged values)
_LAUNCH_PART = {"k_col": slice(0, 3), "k_stage_fwd": slice(3, 5), "k_stage_bwd": slice(5, 8)}


def measured_traffic(workload, kernel, launch, source="llg_kernels.hip"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload (copy-calibrated), or None when there is
    none or it was taken on another kernel source or another tiling of this
    kernel class."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    from paper_2411_19109_amd import profsum
    rec = None
    for line in open(path):
        if line.startswith("{"):
            rec = json.loads(line)
    if not rec or rec.get("kernel_source_sha256") != profsum.kernel_source_hash(source):
        return None
    part = _LAUNCH_PART.get(kernel, slice(None))
    if rec.get("launch") is not None and list(rec["launch"])[part] != list(launch)[part]:
        return None
    for name, v in rec["kernels"].items():
        base = name.split("<")[0]
        if base == kernel or (kernel == "k_col" and base.startswith("k_col")):
            return round(v["hbm_bytes"])
    return None


def _kernel_stats(solver):
    from paper_2411_19109_amd import llg
    kinds = {}
    for k, name in llg.KIND_NAMES.items():
        ms, n, b = solver.profile_read(k)
        if n:
            kinds[name] = dict(ms=ms, launches=n, bytes=b, avg_us=1e3 * ms / n, gbs=b / (ms * 1e-3) / 1e9)
    return kinds


def run_sweep(args):
    """The default bench line: the batched sweep at full length (64 instances x
    --sweep-steps RK4 steps, forward + adjoint gradient per step), the kernel
    averages of the timed steps (HIP events bound to every 7th dispatch of each
    kernel class, on its stream; the roofline from the forward phase, where one
    stream runs alone), the plain path over all 64 instances (one single-instance
    gradient after the other, --plain-steps RK4 steps each: the per-step cost
    of a run does not depend on its length; in its fastest form, per-instance
    launches replayed as HIP graphs, unless --plain-graphs 0), and the oracle
    on the host."""
    import torch
    from paper_2411_19109_amd import llg
    n = args.sweep_steps
    step = SweepStep(n, bool(args.graphs), bool(args.autotune), args.launch_file)
    print(f"[bench] sweep: {len(step.ws)} instances, {step.nodes} nodes, {n} steps, launch {step.launch}, "
          f"setup {step.t_create:.2f} s + tuning {step.t_tune:.2f} s", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    prof = not args.no_kernel_events and _profile_supported(step.batch)
    kinds, kinds_adj = {}, {}
    if prof:
        # every 7th launch of each kernel class carries the event pair (7 is prime to the 4 RK4 stages,
        # so every stage is sampled); bracketing all of them costs the sweep about 4 %
        step.batch.profile(True, stride=7)
    torch.cuda.synchronize()

    def collect(into):
        for name, v in _kernel_stats(step.batch).items():
            acc = into.setdefault(name, dict(ms=0.0, launches=0, bytes=0.0))
            acc["ms"] += v["ms"]
            acc["launches"] += v["launches"]
            acc["bytes"] += v["bytes"]

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        psis, J = step.forward()
        if prof:
            # the forward runs on one stream: its launches are timed alone (reading waits for it to end).
            # In the adjoint the recompute stream overlaps the transposes, and an event pair there also
            # times the other stream's kernels sharing the CUs; those averages are reported apart.
            collect(kinds)
        g = step.backward(psis)
        ev[i + 1].record()
        if prof:
            collect(kinds_adj)
        print(f"[bench] timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    if prof:
        step.batch.profile(False)
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    rate_b = step.nodes * n / tb
    print(f"[bench] batched: {tb * 1e3:.1f} ms per sweep gradient (median {np.median(per_step):.1f} ms), "
          f"{rate_b:.4g} cell-steps/s", file=sys.stderr, flush=True)
    roofline = None
    if kinds:
        for phase, kk in (("forward", kinds), ("adjoint (two streams)", kinds_adj)):
            for name, v in kk.items():
                v["avg_us"] = 1e3 * v["ms"] / v["launches"]
                v["gbs"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9
                print(f"[bench] batched {phase} {name}: {v['launches']} timed launches, avg {v['avg_us']:.2f} us, "
                      f"{v['gbs']:.1f} GB/s algorithmic", file=sys.stderr, flush=True)
        dom = max(kinds, key=lambda k: kinds[k]["ms"])
        d = kinds[dom]
        roofline = dict(bound="hbm", achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(d["gbs"] / HBM_PEAK_GBS, 5),
                        traffic=measured_traffic(SWEEP_NAME, dom, step.launch), kernel=dom,
                        avg_launch_us=round(d["avg_us"], 3), bytes_per_launch=round(d["bytes"] / d["launches"]),
                        timed="forward phase (one stream), every 7th launch")
    J_mean = float(J.double().mean().item())
    del g
    rate_p, tp, n_plain, nplain_steps = None, None, 0, args.plain_steps
    if nplain_steps > 0:
        t_setup = time.perf_counter()
        plain, nodes_p = sweep_plain(nplain_steps, len(step.ws), bool(args.plain_graphs), bool(args.autotune))
        for p in plain:  # first call of each instance (its graphs are captured here when graphs are on)
            p()
        torch.cuda.synchronize()
        print(f"[bench] plain: {len(plain)} single-instance handles ready in {time.perf_counter() - t_setup:.1f} s",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        for p in plain:
            p()
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        n_plain = len(plain)
        rate_p = nodes_p * nplain_steps / tp
        print(f"[bench] plain: {tp * 1e3:.1f} ms for {n_plain} sequential instances x {nplain_steps} steps, "
              f"{rate_p:.4g} cell-steps/s", file=sys.stderr, flush=True)
        for p in plain:
            p.solver.close()
        del plain
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_sweep(n, args.cpu_budget)
        print(f"[bench] cpu baseline: {cpu['value']:.4g} cell-steps/s on {cpu['cores']} cores "
              f"({cpu['one_core_value']:.4g} on one); {cpu['sample']}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": rate_b,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tb * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SWEEP_NAME if n == 10000 else f"yig_demux_sweep_64x_{n}steps_grad",
                   "instances": len(step.ws), "nodes": step.nodes, "rk4_steps": n, "checkpoint": "sqrt",
                   "grad_ms": round(tb * 1e3, 3), "grad_ms_median": round(float(np.median(per_step)), 3),
                   "plain_cell_steps_per_s": rate_p, "plain_instances_timed": n_plain,
                   "plain_rk4_steps_per_instance": nplain_steps if n_plain else None,
                   "batched_over_plain": rate_b / rate_p if rate_p else None, "hip_graphs": bool(args.graphs),
                   "plain_hip_graphs": bool(args.plain_graphs) if n_plain else None,
                   "launch": list(step.launch), "objective_J_mean": J_mean,
                   "setup_s": {"create": round(step.t_create, 3), "launch_tuning": round(step.t_tune, 3)}},
        "roofline": roofline,
        "kernels": {"forward": {k: dict(avg_us=round(v["avg_us"], 2), gbs=round(v["gbs"], 1)) for k, v in kinds.items()},
                    "adjoint_two_streams": {k: dict(avg_us=round(v["avg_us"], 2), gbs=round(v["gbs"], 1))
                                            for k, v in kinds_adj.items()}} if kinds else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_probe(args):
    """HBM-scale measurement of the fused step: a batch of 4 YIG films of
    1024x1024 nodes (FP32 state, spectra and stage buffers ~0.5 GB, beyond the
    256 MB last-level cache), forward RK4 steps only; the roofline object is the
    forward row kernel (fields + LL RHS + RK4 stage + row FFTs)."""
    import torch
    from paper_2411_19109_amd import llg, workloads as wl
    n = args.n_steps or 20
    ws = [wl.yig_film_probe(seed=5 + k, n_steps=n) for k in range(4)]
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float32, device=dev)
    b = llg.Batch([w.problem for w in ws], dtype="f32", max_steps=n)
    if args.launch_file and os.path.exists(args.launch_file):
        b.set_launch_config(*[int(v) for v in open(args.launch_file).read().split()])
        launch = b.launch_config()
    else:
        launch = b.autotune() if args.autotune else b.launch_config()
        if args.launch_file:
            with open(args.launch_file, "w") as fh:
                fh.write(" ".join(str(v) for v in launch) + "\n")
    psis = [t(w.psi_fixed) for w in ws]
    m0 = [t(w.m0) for w in ws]
    nodes = sum(w.problem.n for w in ws)
    print(f"[bench] probe: {len(ws)} x {ws[0].problem.nx}x{ws[0].problem.ny}, {nodes} nodes, {n} steps, "
          f"launch {launch}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        b.forward(psis, m0, n, want_m=False)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        b.forward(psis, m0, n, want_m=False)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    name = "yig_film_probe_4x1024x1024_forward"
    roofline, kinds = None, {}
    if not args.no_kernel_events and _profile_supported(b):
        b.profile(True)
        b.forward(psis, m0, n, want_m=False)
        torch.cuda.synchronize()
        b.profile(False)
        kinds = _kernel_stats(b)
        for kn, v in kinds.items():
            print(f"[bench] probe {kn}: {v['launches']} launches, avg {v['avg_us']:.2f} us, "
                  f"{v['gbs']:.1f} GB/s algorithmic", file=sys.stderr, flush=True)
        d = kinds["k_stage_fwd"]
        roofline = dict(bound="hbm", achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(d["gbs"] / HBM_PEAK_GBS, 5), traffic=measured_traffic(name, "k_stage_fwd", launch),
                        kernel="k_stage_fwd", avg_launch_us=round(d["avg_us"], 3),
                        bytes_per_launch=round(d["bytes"] / d["launches"]))
    out = {
        "metric": "LLG cell-steps/s forward",
        "value": nodes * n / sec,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "nodes": nodes, "rk4_steps": n, "launch": list(launch)},
        "roofline": roofline,
        "kernels": {k: dict(avg_us=round(v["avg_us"], 2), gbs=round(v["gbs"], 1)) for k, v in kinds.items()},
    }
    print(json.dumps(out), flush=True)


def run_adaptive(args):
    """The particle gradient with adaptive Dormand-Prince steps over the same
    physical time as the fixed-step run (2000 x 50 fs = 100 ps), FP32, error
    tolerance 1e-5: adaptive forward, energy objective, adjoint of the
    accepted steps, chain to dJ/dphi.  The forward keeps every accepted
    step's stages for the adjoint (a 4.3 GB store); the recomputing mode is
    timed beside it."""
    import torch
    from paper_2411_19109_amd import llg, workloads as wl
    w = wl.permalloy_particle()
    dev = torch.device("cuda:0")
    t_end = w.n_steps * w.problem.dt
    tol = 1e-5
    s = llg.Solver(w.problem, dtype="f32", max_steps=4 * w.n_steps, design=w.design)
    if args.launch_file and os.path.exists(args.launch_file):
        s.set_launch_config(*[int(v) for v in open(args.launch_file).read().split()])
        launch = s.launch_config()
    else:
        launch = s.autotune()
        if args.launch_file:
            with open(args.launch_file, "w") as fh:
                fh.write(" ".join(str(v) for v in launch) + "\n")
    s.set_keep_stages(True)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float32, device=dev)
    phi, psif, m0 = t(w.phi), t(w.psi_fixed), t(w.m0)
    obj = llg.make_objective(w.objective, E_ref=wl.energy_reference(w), lam=w.obj_lambda, area=w.obj_area)

    def step():
        psi = s.levelset_to_psi(phi, w.heaviside_a, psif)
        mT, hs, nrej = s.forward_adaptive(psi, m0, t_end, w.problem.dt, tol, tol)
        J, dJdm, dJdpsi_e, _ = s.objective(obj, psi, mT)
        dpsi = s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e)
        return J, s.levelset_vjp(phi, dpsi, w.heaviside_a), hs, nrej
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        J, g, hs, nrej = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    n_acc = len(hs)
    print(f"[bench] adaptive particle: {n_acc} accepted, {nrej} rejected steps (h {hs.min():.3e}..{hs.max():.3e} s), "
          f"{sec * 1e3:.1f} ms per gradient", file=sys.stderr, flush=True)
    # the continuous adjoint (Eqs. 6-7) of the same run beside the discrete one: time of the backward
    # pass alone and the relative L2 gap of dJ/dphi.  Two RK4 sub-steps per interval: the adaptive steps of
    # this stiff run sit at the edge of Dormand-Prince's stability region, beyond RK4's.
    n_sub = 2
    psi = s.levelset_to_psi(phi, w.heaviside_a, psif)
    mT, hs, nrej = s.forward_adaptive(psi, m0, t_end, w.problem.dt, tol, tol)
    _, dJdm, dJdpsi_e, _ = s.objective(obj, psi, mT)
    back = {}
    for key, cont in (("discrete", False), ("continuous", True)):
        s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, continuous=cont, n_sub=n_sub)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            dpsi = s.adjoint_adaptive(psi, dJdm_T=dJdm, dJdpsi_expl=dJdpsi_e, continuous=cont, n_sub=n_sub)
        torch.cuda.synchronize()
        back[key] = ((time.perf_counter() - t0) / max(1, args.steps), s.levelset_vjp(phi, dpsi, w.heaviside_a))
    gd, gc = back["discrete"][1].double(), back["continuous"][1].double()
    gap = float((gc - gd).norm() / gd.norm())
    compare = {"discrete_adjoint_ms": round(back["discrete"][0] * 1e3, 2),
               "continuous_adjoint_ms": round(back["continuous"][0] * 1e3, 2), "continuous_sub_steps": n_sub,
               "continuous_vs_discrete_rel_l2": gap}
    print(f"[bench] adaptive backward pass: discrete {compare['discrete_adjoint_ms']} ms, continuous "
          f"{compare['continuous_adjoint_ms']} ms, dJ/dphi gap {gap:.2e}", file=sys.stderr, flush=True)
    # the same gradient without the stage store: the adjoint recomputes each step's stages (bitwise the same)
    s.set_keep_stages(False)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        _, gr, _, _ = step()
    torch.cuda.synchronize()
    compare["recomputed_stages_ms_per_gradient"] = round((time.perf_counter() - t0) / max(1, args.steps) * 1e3, 2)
    compare["recomputed_stages_bitwise_equal"] = bool(torch.equal(gr, g))
    s.set_keep_stages(True)
    print(f"[bench] adaptive gradient recomputing the stages: {compare['recomputed_stages_ms_per_gradient']} ms "
          f"(kept stages: {sec * 1e3:.1f} ms), bitwise equal: {compare['recomputed_stages_bitwise_equal']}",
          file=sys.stderr, flush=True)
    roofline, kinds = None, {}
    if not args.no_kernel_events and _profile_supported(s):
        s.profile(True)
        step()
        torch.cuda.synchronize()
        s.profile(False)
        kinds = _kernel_stats(s)
        for kn, v in kinds.items():
            print(f"[bench] adaptive {kn}: {v['launches']} launches, avg {v['avg_us']:.2f} us, "
                  f"{v['gbs']:.1f} GB/s algorithmic", file=sys.stderr, flush=True)
        dom = max(kinds, key=lambda k: kinds[k]["ms"])
        d = kinds[dom]
        roofline = dict(bound="hbm", achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(d["gbs"] / HBM_PEAK_GBS, 5), traffic=None, kernel=dom,
                        avg_launch_us=round(d["avg_us"], 3), bytes_per_launch=round(d["bytes"] / d["launches"]))
    N = w.problem.n
    out = {
        "metric": METRIC,
        "value": N * n_acc / sec,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "permalloy_particle_64x64_adaptive_grad", "nodes": [w.problem.nx, w.problem.ny, 1],
                   "t_end_s": t_end, "rtol": tol, "atol": tol, "accepted_steps": n_acc, "rejected_steps": nrej,
                   "fixed_step_equivalent": w.n_steps, "launch": list(launch), "objective_J": float(J.item()),
                   "kept_stages": True, "stage_store_bytes": 11 * (4 * w.n_steps + 1) * 3 * w.problem.n * 4},
        "roofline": roofline,
        "kernels": {k: dict(avg_us=round(v["avg_us"], 2), gbs=round(v["gbs"], 1)) for k, v in kinds.items()},
        "adjoint_compare": compare,
    }
    print(json.dumps(out), flush=True)


# VALU issue rate of the chip: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (one non-packed VALU instruction per lane per clock).  Transcendental
# instructions (sqrt, log2, exp2) issue at half that rate on CDNA 4, so one
# counts as two issue slots.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
# Arithmetic per node-RBF pair of each kernel (plain VALU ops, transcendentals):
# cones: 2 sub, 2 fma, sub, min, max + sqrt; p-norm: 2 sub, 2 fma, sub, max, mul,
# mul, add + sqrt, log2, exp2; VJP: 2 sub, 2 fma, sub, max, fma, fma + sqrt,
# log2, exp2.  Per-node work (loads, coordinates, the node's own log2) is not
# counted: the bound is the pair arithmetic alone.
RBF_PAIR_OPS = {"k_rbf_cones": (7, 1), "k_rbf_pnorm": (9, 3), "k_rbf_vjp": (8, 3)}


def rbf_pair_peak(kernel):
    plain, trans = RBF_PAIR_OPS[kernel]
    return VALU_LANE_OPS / (plain + 2 * trans)


def rbf_step_factory(nx, ny, n_side, dtype="f32", seed=7):
    """One design update of the RBF stage on an nx x ny design region: phi from
    s, dJ/ds from a fixed dJ/dphi, an Adam step on s."""
    import torch
    from paper_2411_19109_amd import llg, workloads as wl
    D = min(nx, ny)
    lay = wl.rbf_layout((0, 0, D), n_side=n_side, holes=4, seed=seed)
    if nx != ny:   # stretch the square array over the whole rectangle
        lay["xc"] = lay["xc"] * (nx / D)
        lay["yc"] = lay["yc"] * (ny / D)
    design = np.ones((ny, nx), np.uint8)
    m = llg.RBFLevelSet(lay["xc"], lay["yc"], lay["c"], lay["p"], design, dtype=dtype)
    s = torch.as_tensor(lay["s"], dtype=torch.float64, device="cuda")
    g = torch.as_tensor(np.random.default_rng(seed).standard_normal(nx * ny), dtype=torch.float64, device="cuda")
    opt = llg.Adam(s.numel(), lr=1e-3)
    work = m.new_work()

    def step():
        phi, pn, _ = m.levelset(s, work=work)
        ds = m.vjp(s, g, pn, work)
        opt.step(s, ds)
        return phi, ds
    return step, lay, m


def rbf_cpu_baseline(budget_s=15.0):
    """The oracle's level set and VJP on a band of rows of the same 1024-wide
    film with the same 400 RBFs, sized to about budget_s of host time."""
    from oracle import rbf as orbf
    from paper_2411_19109_amd import workloads as wl
    lay = wl.rbf_layout((0, 0, 1024), n_side=20, holes=4, seed=7)
    ctr = (lay["xc"], lay["yc"])

    def run(rows):
        design = np.ones((rows, 1024))
        t0 = time.perf_counter()
        phi, dphi, sc = orbf.pnorm_levelset(lay["s"], ctr, lay["c"], lay["p"], design)
        orbf.pnorm_levelset_vjp(lay["s"], ctr, lay["c"], lay["p"], design, np.ones_like(phi), dphi, sc)
        return time.perf_counter() - t0
    rows = 2
    dt = run(rows)
    rows = int(max(2, min(1024, rows * budget_s / max(dt, 1e-3))))
    dt = run(rows)
    pairs = rows * 1024 * lay["xc"].size
    return dict(value=pairs / dt, unit="pairs/s", cores=1, kind="oracle",
                sample=f"float64 NumPy oracle, level set + VJP of {rows} rows x 1024 nodes x {lay['xc'].size} RBFs "
                       f"({dt:.1f} s, one host thread)")


def run_rbf(args):
    """The RBF stage of the design loop (Eqs. 2, 3, renormalisation, VJP, Adam)
    at scale: a 1024x1024-node design region with the paper's 20x20 RBF array
    (FP32), plus the paper's own sizes (the particle's 64x64 mesh and the
    demultiplexer's 256x96 grid with its 60x60 design square) timed per update."""
    import torch
    from paper_2411_19109_amd import llg
    nx = ny = 1024
    step, lay, m = rbf_step_factory(nx, ny, 20)
    n = lay["xc"].size
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    pairs = nx * ny * n
    print(f"[bench] rbf {nx}x{ny}, {n} RBFs: {sec * 1e6:.1f} us per update "
          f"(events {e0.elapsed_time(e1) / args.steps * 1e3:.1f} us)", file=sys.stderr, flush=True)

    # the paper's sizes, one update each (launch-bound at these sizes)
    small = {}
    from paper_2411_19109_amd import workloads as wl
    sizes = {"particle_64x64": (64, 64, (0, 0, 64)),
             "demux_256x96": (256, 96, wl.yig_demux(n_steps=10).extra["box"])} if args.rbf_paper_sizes else {}
    for name, (sx, sy, box) in sizes.items():
        sl = wl.rbf_layout(box, n_side=20, holes=4, seed=1)
        d2 = np.zeros((sy, sx), np.uint8)
        d2[box[1]:box[1] + box[2], box[0]:box[0] + box[2]] = 1
        sm = llg.RBFLevelSet(sl["xc"], sl["yc"], sl["c"], sl["p"], d2, dtype="f32")
        ss = torch.as_tensor(sl["s"], dtype=torch.float64, device="cuda")
        gg = torch.ones(sx * sy, dtype=torch.float64, device="cuda")
        opt = llg.Adam(ss.numel(), lr=1e-3)
        wk = sm.new_work()

        def upd():
            phi, pn, _ = sm.levelset(ss, work=wk)
            opt.step(ss, sm.vjp(ss, gg, pn, wk))
        for _ in range(3):
            upd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            upd()
        torch.cuda.synchronize()
        small[name] = round((time.perf_counter() - t0) / 50 * 1e6, 1)
        print(f"[bench] rbf {name}: {small[name]} us per update", file=sys.stderr, flush=True)

    roofline, kinds = None, {}
    if not args.no_kernel_events and os.environ.get("ROCPROF_COUNTER_COLLECTION") is None:
        llg.rbf_profile(True)
        step()
        torch.cuda.synchronize()
        llg.rbf_profile(False)
        for k, kn in llg.RBF_KIND_NAMES.items():
            ms, nl, pr = llg.rbf_profile_read(k)
            if nl:
                rate = pr / (ms * 1e-3)
                peak = rbf_pair_peak(kn)
                kinds[kn] = dict(avg_us=round(1e3 * ms / nl, 2), gpairs=round(rate / 1e9, 1),
                                 peak_gpairs=round(peak / 1e9, 1), frac=round(rate / peak, 4))
                print(f"[bench] {kn}: {nl} launches, avg {1e3 * ms / nl:.1f} us, {rate / 1e9:.1f} Gpairs/s "
                      f"({rate / peak:.3f} of the ALU bound {peak / 1e9:.0f})", file=sys.stderr, flush=True)
        dom = max(kinds, key=lambda k: kinds[k]["avg_us"])
        d = kinds[dom]
        roofline = dict(bound="alu", achieved=d["gpairs"], peak=d["peak_gpairs"], unit="Gpairs/s", frac=d["frac"],
                        traffic=measured_traffic(f"rbf_levelset_film_{nx}x{ny}_{n}rbf", dom, None, "llg_rbf.hip"),
                        kernel=dom, avg_launch_us=d["avg_us"], pairs_per_launch=pairs,
                        ops_per_pair=dict(zip(("plain", "transcendental"), RBF_PAIR_OPS[dom])))
    cpu = None
    if not args.no_cpu:
        cpu = rbf_cpu_baseline(args.cpu_budget)
        print(f"[bench] cpu baseline: {cpu['sample']}", file=sys.stderr, flush=True)
    out = {
        "metric": "RBF level set + VJP + Adam: node-RBF pairs/s",
        "value": pairs / sec,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rbf_levelset_film_{nx}x{ny}_{n}rbf", "nodes": nx * ny, "n_rbf": n, "p": lay["p"],
                   "update_us": round(sec * 1e6, 1), "paper_sizes_us_per_update": small},
        "roofline": roofline,
        "kernels": kinds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
