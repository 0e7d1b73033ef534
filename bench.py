#!/usr/bin/env python3
"""Benchmark of the SMAME step on one MI355X.

Default workload: 3D periodic Taylor-Green vortex, 256^3 nodes, FP32 with
drho storage, u0 = 0.05, Re = 1600 on a 2 pi box, one SMAME step per
"step" (the fused 2.5D z-march kernel).  Prints ONE JSON line with MLUPS,
HBM GB/s against the 8 TB/s peak, the roofline record of the step kernel
and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="tgv3d_256",
                    choices=["tgv3d_256", "tgv2d_64", "drop_shear_1024", "drop_spreading_96", "batch512",
                             "pipe_axisym_4096x2048", "drop_axisym_2048x1024"])
    ap.add_argument("--no-closure", action="store_true",
                    help="skip the closure, drop-in-shear and batch-sweep objects of the default workload's line")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--batch-mode", type=int, default=0, choices=(0, 1),
                    help="batch512: 0 one workgroup per item, 1 persistent work queue")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-only", action="store_true",
                    help="time only the plain copy kernel (bandwidth / counter calibration)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    return ap.parse_args()


def copy_bandwidth(mib: int, reps: int = 20):
    """Achieved rate of the library's plain copy kernel: bytes read + written
    per second for a `mib` MiB buffer (read mib, write mib per launch)."""
    import torch
    from paper_2012_03525_amd import acm
    n = mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    s = torch.cuda.current_stream()
    for _ in range(3):
        acm.stream_copy(dst, src, n, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        acm.stream_copy(dst, src, n, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_per_launch": 2 * n, "avg_launch_us": round(ms * 1e3, 2), "gbs": round(2 * n / (ms * 1e-3) / 1e9, 1)}


def graph_chunk_for(steps: int, cap: int = 100) -> int:
    """Largest even graph chunk <= cap that divides the even part of `steps`,
    so that every timed step (but the last of an odd count) runs inside a
    captured graph; the library captures both parities' graphs at init."""
    even = steps - steps % 2
    for c in range(min(cap, even), 1, -1):
        if c % 2 == 0 and even % c == 0:
            return c
    return 2


def workload(name, tile, chunk=100):
    from paper_2012_03525_amd import acm, inputs
    if name == "tgv3d_256":
        n, u0 = 256, 0.05
        nu = u0 * (n / (2 * math.pi)) / 1600.0
        cfg = acm.make_config(3, n, n, n, nu=nu, precision="f32", tile=tile, graph_chunk=chunk)
        st = inputs.tgv3d(n, u0)
        meta = {"workload": "3D periodic Taylor-Green vortex 256^3, FP32 drho storage",
                "grid": [n, n, n], "u0": u0, "Re": 1600, "nu_lattice": nu, "steps_of_case": 2000}
        bytes_per_lup = 32  # read drho,u,v,w + write drho,u,v,w (FP32)
        kernel = "step3d_rows_kernel"
    elif name == "tgv2d_64":
        n = 64
        cfg = acm.make_config(2, n, n, nu=0.01, precision="f64", tile=tile, graph_chunk=chunk)
        st = inputs.tgv2d(n, 0.01, noise=1e-6)
        meta = {"workload": "2D periodic Taylor-Green vortex 64^2, FP64", "grid": [n, n], "u0": 0.01, "nu": 0.01}
        bytes_per_lup = 48
        kernel = "step2d_kernel"
    elif name == "pipe_axisym_4096x2048":
        # axisymmetric pipe (x axial, periodic; y radial: axis, wall at r = R = 2048): start-up of the
        # axially forced flow from a perturbed profile; g sets the Poiseuille centre speed to 0.05
        nxa, R, nu = 4096, 2048, 0.05
        g = 4.0 * nu * 0.05 / (R * R)
        cfg = acm.make_config(2, nxa, R, nu=nu, g=(g, 0.0, 0.0), precision="f32", bc=(0, 0, 2, 1, 0, 0),
                              axisym=True, tile=tile, graph_chunk=chunk)
        st = inputs.pipe_state(nxa, R, seed=3)
        meta = {"workload": "axisymmetric pipe flow 4096 (axial) x 2048 (radial), FP32 drho storage",
                "grid": [nxa, R], "nu": nu, "g": g}
        bytes_per_lup = 24  # read drho,u,v + write drho,u,v (FP32)
        kernel = "axisym2d_kernel"
    elif name == "drop_axisym_2048x1024":
        # axisymmetric two-phase: a drop (sphere) of radius 256 on the axis of an axially periodic
        # 2048 x 1024 domain with a symmetry rim, relaxing under surface tension
        nxa, nr, R, W = 2048, 1024, 256.0, 4.0
        cfg = acm.make_config(2, nxa, nr, nu=0.1, precision="f32", bc=(0, 0, 2, 2, 0, 0), axisym=True,
                              two_phase=True, sigma=0.01, width=W, mobility=0.1, tile=tile, graph_chunk=chunk)
        st = inputs.drop_on_axis(nxa, nr, R, W)
        meta = {"workload": "axisymmetric two-phase drop on the axis 2048 (axial) x 1024 (radial), FP32",
                "grid": [nxa, nr], "R": R, "W": W, "sigma": 0.01, "mobility": 0.1, "nu": 0.1}
        bytes_per_lup = 32  # read drho,u,v,phi + write them (FP32)
        kernel = "twophase2d_kernel (axisymmetric)"
    elif name == "drop_spreading_96":
        # drop spreading on a wall (Sec. 3.6): N_L = 32, c = 10, Re = 100 (Oh = 0.1), Cn = 0.1,
        # Pe = 8000, theta = 60 degrees; [0,3]^3 with symmetry planes at the sides, walls at z = 0, 3
        NL, c, Re, Cn, Pe, theta = 32, 10.0, 100.0, 0.1, 8000.0, 60.0
        n = 3 * NL
        nu = NL / (c * Re)
        sigma = NL / (c * c * Re)
        W = Cn * NL
        M = NL * NL / (Pe * nu)
        wet = [0.0] * 6
        wet[4] = math.cos(math.radians(theta))
        cfg = acm.make_config(3, n, n, n, nu=nu, precision="f32", bc=(2, 2, 2, 2, 1, 1), two_phase=True,
                              sigma=sigma, width=W, mobility=M, tile=tile, graph_chunk=chunk, wet_cos=wet)
        st = inputs.drop_on_wall_3d(n, n, n, float(NL), W, center=(0.0, 0.0, 0.0))
        meta = {"workload": "3D drop spreading on a wall 96^3 (N_L = 32, theta = 60 deg), FP32", "grid": [n, n, n],
                "N_L": NL, "c": c, "Re": Re, "Cn": Cn, "Pe": Pe, "theta_deg": theta, "nu": nu, "sigma": sigma,
                "mobility": M}
        bytes_per_lup = 40  # read drho,u,v,w,phi + write them (FP32), the fused minimum
        kernel = "twophase3d step (3 launches)"
    else:
        n = 1024
        wu = [[0.0] * 3 for _ in range(6)]
        wu[2] = [-0.02, 0, 0]
        wu[3] = [0.02, 0, 0]
        # nu = 1/6: at nu = 0.1 this drop diverges after about 2000 steps (oracle and GPU alike)
        cfg = acm.make_config(2, n, n, nu=1.0 / 6.0, precision="f32", bc=(0, 0, 1, 1, 0, 0), wall_u=wu,
                              two_phase=True, sigma=0.01, width=4.0, mobility=0.02, tile=tile, graph_chunk=chunk)
        st = inputs.drop_in_shear(n, n, 128.0, 4.0, 0.02)
        meta = {"workload": "2D two-phase drop in simple shear 1024^2, FP32", "grid": [n, n], "R": 128, "W": 4,
                "mobility": 0.02, "u_wall": 0.02, "nu": round(1.0 / 6.0, 6), "sigma": 0.01, "steps_of_case": 20000}
        bytes_per_lup = 32
        kernel = "twophase2d_kernel"
    return cfg, st, meta, bytes_per_lup, kernel


def measured_traffic(name):
    """HBM bytes per launch of the workload's dominant kernel from the
    committed counter runs (profiles/traffic.json), or None when the kernel
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[name]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha1()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha1"]:
        return None
    return int(1024 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]))


def batch_sweep(mode: int):
    """The 512-case sweep, one batched launch per step (FP32, autotuned
    tiles, 500-step graph chunks): aggregate MLUPS over the whole job and the
    p50 / p99 case completion times."""
    import numpy as np
    from paper_2012_03525_amd import acm, inputs
    cases = inputs.batch_cases(512, seed=4)
    cfgs, states = [], []
    for c in cases:
        wu = [[0.0] * 3 for _ in range(6)]
        bc = (0, 0, 0, 0, 0, 0)
        if c.kind == "cavity":
            bc = (1, 1, 1, 1, 0, 0)
            wu[3] = [c.u_ref, 0.0, 0.0]
        cfgs.append(acm.make_config(2, c.n, c.n, nu=c.nu, precision="f32", bc=bc, wall_u=wu))
        states.append(c.state)
    print(f"[bench] batch: {len(cases)} cases, {sum(c.n * c.n for c in cases)} nodes", file=sys.stderr, flush=True)
    b = acm.Batch(cfgs, states, [c.nsteps for c in cases], chunk=500, mode=mode)
    b.run()
    ms, lups = b.timing()
    st = [b.status(i) for i in range(len(cases))]
    done = np.array([s["done_ms"] for s in st if s["state"] == acm.BATCH_FINISHED])
    diverged = sum(1 for s in st if s["state"] != acm.BATCH_FINISHED)
    b.close()
    return {"cases": len(cases), "lattice_updates": int(lups), "wall_ms": round(ms, 2),
            "mlups": round(lups / (ms * 1e-3) / 1e6, 1), "gbs": round(24 * lups / (ms * 1e-3) / 1e9, 1),
            "steps": int(max(c.nsteps for c in cases)),
            "p50_ms": round(float(np.percentile(done, 50)), 2), "p99_ms": round(float(np.percentile(done, 99)), 2),
            "finished": int(done.size), "diverged": diverged}


def run_batch(a, copy):
    """The 512-case sweep as its own bench line."""
    r = batch_sweep(a.batch_mode)
    out = {
        "metric": "MLUPS + HBM GB/s vs peak; learned-coarse vs plain-fine time at <=2% L2 err",
        "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": r["steps"],
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched sweep: 512 2D cases n in {32..256}, half periodic TGV / half lid-driven "
                               "cavity, Re log-uniform [100, 5000], FP32, one launch per step, 500-step graph chunks",
                   "launch": ["one workgroup per item", "persistent work queue"][a.batch_mode],
                   "cases": r["cases"], "lattice_updates": r["lattice_updates"], "parallelism": "single GPU"},
        "wall_ms": r["wall_ms"],
        "case_completion_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"], "finished": r["finished"],
                               "diverged": r["diverged"]},
        "roofline": {"bound": "hbm", "kernel": ["batch_grid_kernel", "batch_step_kernel"][a.batch_mode],
                     "achieved": r["gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(r["gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_lup": 24, "copy_kernel_gbs": copy["gbs"]},
    }
    print(json.dumps(out), flush=True)


def drop_shear_timing(steps: int = 1000, warmup: int = 50):
    """The 2D two-phase drop in shear (1024^2, FP32): time per step of the
    fused two-phase launch, graph-launched, HIP events on the solver's stream."""
    import torch
    from paper_2012_03525_amd import acm
    cfg, st, meta, bpl, kname = workload("drop_shear_1024", 0, 100)
    s = acm.Solver(cfg, st)
    s.run(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    d = s.diagnostics()
    s.close()
    nodes = cfg.nx * cfg.ny
    gbs = bpl * nodes / (ms * 1e-3) / 1e9
    return {"workload": meta["workload"], "kernel": kname, "steps": steps, "us_per_step": round(ms * 1e3, 3),
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "gbs_algorithmic": round(gbs, 1),
            "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4), "nonfinite": d["nonfinite"]}


def closure_timing(steps: int = 2000):
    """Closure step (coarse 256^2 SMAME step + fused network correction) against
    the four fine 1024^2 steps it replaces, graph-launched; the network's
    accuracy comes from the closure experiment, not from this timing."""
    from paper_2012_03525_amd import closure_experiment
    t = closure_experiment.step_timing("full", steps=steps, log=lambda m: None)
    return {"fine_1024_x4_us": round(t["fine_steps_per_coarse_step_us"], 2),
            "closure_256_step_us": round(t["closure_step_us"], 2),
            "plain_coarse_256_step_us": round(t["plain_coarse_step_us"], 2),
            "closure_256_two_launch_step_us": round(t["closure_separate_launch_step_us"], 2),
            "adjoint_256_step_us": round(t["adjoint_step_us"], 2),
            "speedup_vs_fine": round(t["fine_steps_per_coarse_step_us"] / t["closure_step_us"], 3)}


def closure_evaluation(train_seeds=(0, 50), eval_seeds=(2000, 2010)):
    """The learned-coarse vs plain-fine comparison, live and bounded: the
    full preset's recipe (256^2 coarse / 1024^2 fine, 10,000 coarse steps)
    trained on fewer seeds and evaluated on ten held-out seeds; time to
    solution of the gated closure run (gates and fallbacks included) against
    40,000 plain fine steps, and the largest relative L2 velocity error over
    the gates.  The 50-seed evaluation is the closure experiment's."""
    from paper_2012_03525_amd import closure_experiment
    t0 = time.perf_counter()
    r, _ = closure_experiment.run_experiment("full", log=lambda m: None, train_seeds=train_seeds,
                                             eval_seeds=eval_seeds)
    return {"train_seeds": list(train_seeds), "eval_seeds": list(eval_seeds),
            "time_to_solution_closure_ms": round(r["mean_t_closure_s"] * 1e3, 2),
            "time_to_solution_fine_ms": round(r["mean_t_fine_s"] * 1e3, 2),
            "speedup": round(r["mean_t_fine_s"] / r["mean_t_closure_s"], 3),
            "max_rel_l2_err_closure": round(r["max_err_closure_max"], 5),
            "gate_trips": r["gate_trips"],
            "seeds_within_2pct_and_faster": r["seeds_closure_within_2pct_and_faster"],
            "wall_s": round(time.perf_counter() - t0, 1)}


def cpu_baseline(name, cfg, st, budget_s):
    """Time the FP64 CPU oracle (single thread) on a bounded sample of the
    same workload: whole-grid steps until about budget_s seconds pass."""
    import oracle
    oracle.build(force=False)
    p = oracle.Params(dim=cfg.dim, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, dx=cfg.dx, dt=cfg.dt, nu=cfg.nu,
                      cs=(cfg.cs if cfg.cs > 0 else cfg.dx / (cfg.dt * math.sqrt(3))), rho0=cfg.rho0,
                      sat_rho=cfg.sat_rho, sat_mom=cfg.sat_mom, g=[cfg.g[a] for a in range(3)],
                      bc=list(cfg.bc), wall_u=[[cfg.wall_u[f][a] for a in range(3)] for f in range(6)],
                      two_phase=bool(cfg.two_phase), sigma=cfg.sigma, width=cfg.width, mobility=cfg.mobility,
                      wet_cos=[cfg.wet_cos[f] for f in range(6)], axisym=bool(cfg.axisym))
    nodes = cfg.nx * cfg.ny * (cfg.nz if cfg.dim == 3 else 1)
    t0 = time.perf_counter()
    steps = 0
    s = st
    while True:
        s = oracle.step(p, s)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 1000:
            break
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": nodes * steps / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} whole-grid FP64 steps of the same workload ({nodes} nodes) in {el:.1f} s, "
                      f"single thread, host has {os.cpu_count()} logical CPUs ({model})"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2012_03525_amd import acm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    acm.lib()
    if a.copy_only:
        print(json.dumps({"copy": copy_bandwidth(a.copy_mib)}), flush=True)
        return
    if a.workload == "batch512":
        copy = copy_bandwidth(1024)
        print(f"[bench] plain copy kernel: {copy['gbs']} GB/s", file=sys.stderr, flush=True)
        run_batch(a, copy)
        return
    chunk = graph_chunk_for(a.steps)
    cfg, st, meta, bpl, kname = workload(a.workload, a.tile, chunk)
    solver = acm.Solver(cfg, st)
    nodes = cfg.nx * cfg.ny * (cfg.nz if cfg.dim == 3 else 1)
    # The copy-bandwidth calibration runs right before the warm-up steps: a
    # chip coming out of idle (state upload, graph capture) runs its first
    # ~200 launches of the step 10-30 % slower while its clocks settle, and
    # about 0.1 s of sustained HBM traffic brings it to the state the step
    # then runs in, for the copy ceiling and the step alike.
    copy = copy_bandwidth(1024, reps=250)
    print(f"[bench] plain copy kernel: {copy['gbs']} GB/s", file=sys.stderr, flush=True)
    print(f"[bench] {meta['workload']}: warmup {a.warmup}", file=sys.stderr, flush=True)
    solver.run(a.warmup)
    torch.cuda.synchronize()
    stream = solver.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    solver.run(a.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / a.steps
    mlups = nodes / (ms_per_step * 1e-3) / 1e6
    gbs = bpl * nodes / (ms_per_step * 1e-3) / 1e9
    d = solver.diagnostics()
    print(f"[bench] {a.steps} steps: {gpu_ms:.2f} ms GPU, {wall*1e3:.2f} ms wall, {mlups:.0f} MLUPS, "
          f"{gbs:.0f} GB/s, nonfinite={d['nonfinite']}", file=sys.stderr, flush=True)
    out = {
        "metric": "MLUPS + HBM GB/s vs peak; learned-coarse vs plain-fine time at <=2% L2 err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.precision == acm.F32 else "f64",
        "data": "synthetic",
        "config": dict(meta, parallelism="single GPU"),
        "hbm_gbs_algorithmic": round(gbs, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(a.workload),
            "bytes_per_lup": bpl,
            "lups_per_launch": nodes,
            "avg_launch_us": round(ms_per_step * 1e3, 3),
            "launch_timing": f"HIP events on the library's stream around {a.steps} step launches "
                             f"(graphs of {chunk} launches each)",
            "copy_kernel_gbs": copy["gbs"],
            "frac_of_copy": round(gbs / copy["gbs"], 4),
        },
        "state_check": {"nonfinite": d["nonfinite"], "ke": d["ke"], "step": d["step"]},
    }
    solver.close()
    if a.workload == "tgv3d_256" and not a.no_closure:
        print("[bench] closure step timing...", file=sys.stderr, flush=True)
        out["closure"] = closure_timing()
        print("[bench] closure train + evaluation (10 held-out seeds)...", file=sys.stderr, flush=True)
        out["closure"]["evaluation"] = closure_evaluation()
        print("[bench] 2D two-phase drop in shear 1024^2...", file=sys.stderr, flush=True)
        out["drop_shear"] = drop_shear_timing()
        print("[bench] 512-case batch sweep (one workgroup per item)...", file=sys.stderr, flush=True)
        out["batch"] = dict(batch_sweep(0), launch="one workgroup per item", bytes_per_lup=24)
    if not a.no_cpu:
        print("[bench] CPU oracle baseline...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.workload, cfg, st, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
