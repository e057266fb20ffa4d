"""Benchmark of the UGKWP-LTS hot path on one MI355X.

Workload (the one the metric is quoted on): hypersonic flow past a cylinder,
argon-like VHS gas (omega 0.81, Pr 2/3), Ma 15, Kn 0.01 on the radius,
isothermal diffuse wall T_w/T_inf = 0.2, structured O-grid 200 x 150 to 15 R
with first-layer height 1e-4 R, N_ref 400, local time stepping, FP64.  Inputs
are synthetic (uniform freestream start), resident in HBM before timing.

A step is one whole UGKWP-LTS step (cell preparation, resampling, transport
with LTS scaling, tally and re-sort, wave fluxes, update, wall quantities).
Prints one JSON line.  --gpus N > 1 is not supported (one GPU per process;
the domain-decomposition design is described with the code).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one particle update: read and write one particle
# record (2D: x, y, u_x, u_y, u_z, m, pid, cell = 60 B in FP64; 40 B with
# FP32 cell-relative positions and velocities).  The transport, the kernel
# that moves every particle, is held against it per launch.
TRANSPORT_BYTES = {"f64": 120.0, "mixed": 80.0}
TRANSPORT_BYTES_PER_PARTICLE = TRANSPORT_BYTES["f64"]
TRAFFIC_FILES = {"f64": os.path.join(ROOT, "profiles", "step_traffic_cylinder.json"),
                 "mixed": os.path.join(ROOT, "profiles", "step_traffic_cylinder_mixed.json")}
KERNEL_SRC = os.path.join(ROOT, "paper_2607_09552_amd", "csrc", "kernels.hip")


def workload(kn=0.01, lts=1):
    return workloads.cylinder(n_theta=200, n_r=150, Ma=15.0, Kn=kn, omega=0.81, Pr=2.0 / 3.0, Tw=0.2, n_ref=400,
                              lts=lts, seed=1)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(precision="f64"):
    """HBM bytes per transported particle (FETCH_SIZE + WRITE_SIZE, each
    scaled by what the counter reads for the library's streaming copy of
    known size), per kernel and for the whole step, from the committed
    rocprofv3 counter summary if it was taken on the current kernel source;
    else None."""
    try:
        with open(TRAFFIC_FILES[precision]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"host_cpu": model, "nproc": avail, "cpu_count": os.cpu_count()}


def oracle_shock(steps=2000):
    """The oracle over the whole 1D shock run (100 cells, N_ref 200, LTS,
    FP64, seed 1): particle updates/s and cell-steps/s on one core."""
    import oracle
    w = workloads.shock1d()
    o = oracle.Oracle(w)
    n_upd = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step(1)
        n_upd += o.counts()[1]["total"]
    dt = time.perf_counter() - t0
    o.close()
    return {"workload": "1D Ma 3 shock, 100 cells, N_ref 200, LTS, FP64", "steps": steps, "seconds": dt,
            "particle_updates_per_s": n_upd / dt, "cell_steps_per_s": w["n_cells"] * steps / dt}


def cpu_baseline(w, state, steps):
    """The CPU oracle, as it stands (serial, one thread), on `steps` steps of
    the same workload from the state the GPU run reached (fields, particles
    and step counter loaded into the oracle)."""
    import oracle
    W, p, step0 = state
    o = oracle.Oracle(w)
    o.set_fields(W)
    o.set_particles(p["pid"], p["cell"], p["m"], p["x"], p["u"], p["ei"])
    o.set_step(step0)
    n_upd = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step(1)
        n_upd += o.counts()[1]["total"]
    dt = time.perf_counter() - t0
    o.close()
    out = dict(value=n_upd / dt, unit="particle updates/s", cores=1, kind="oracle",
               sample=f"{steps} steps of the same cylinder workload from the GPU state after step {step0} "
                      f"({len(p['pid'])} retained particles), {n_upd} particle updates in {dt:.1f} s, 1 thread",
               cell_steps_per_s=w["n_cells"] * steps / dt)
    out.update(host_info())
    out["shock1d_full_run"] = oracle_shock()
    return out


def copy_probe(gib=1.0, reps=5):
    """The library's streaming copy (k_stream_copy) of known size, for
    scaling rocprofv3 byte counters and as the attainable HBM rate (bytes
    read + written per second), over a few grid sizes; torch's copy_ beside
    it for comparison."""
    import torch
    from paper_2607_09552_amd import stream_copy
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    runs = {}
    for blocks in (0, 4 * cus, 16 * cus, 32 * cus, (n * 8 // 16 + 255) // 256):
        ms = stream_copy(b, a, reps=reps, blocks=blocks)
        runs[str(blocks)] = {"ms_per_copy": ms, "GBps": 2 * n * 8 / (ms * 1e-3) / 1e9}
    assert torch.equal(a, b)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    best = max(v["GBps"] for v in runs.values())
    print(json.dumps({"copy_probe_bytes_each_way": n * 8, "reps": reps, "compute_units": cus,
                      "stream_copy_by_grid": runs, "stream_copy_best_GBps": best,
                      "torch_copy_GBps": 2 * n * 8 / (ms * 1e-3) / 1e9}))


def time_to_residual(a):
    """Wall clock to the first step n >= 100 with r_avg < target (the
    residual of the running mean density), from the uniform freestream or
    from the learned warm start (--warm-start: coarse solve, features,
    network, decode; its time is part of the value).  The fine solver's
    init is excluded in both.  Prints progress and one JSON line."""
    import numpy as np
    import torch
    from paper_2607_09552_amd import Solver
    w = workload(a.kn) if a.workload == "cylinder" else workloads.flat_plate(seed=1)
    w["dt_source"] = {"initial": 0, "freestream": 1}[a.dt_source]
    W0, ws_info = None, None
    if a.warm_start:
        if a.workload != "cylinder":
            raise SystemExit("--warm-start: the warm-start network is trained on the cylinder")
        from paper_2607_09552_amd import warmstart as ws
        mlp = ws.MLP.load()
        torch.cuda.synchronize()
        W0, ws_info = ws.warm_start(15.0, a.kn, 0.2, mlp=mlp, wl=w)
        print(f"# warm start {ws_info['seconds']:.2f} s (coarse solve {ws_info['coarse_seconds']:.2f} s)",
              file=sys.stderr, flush=True)
    s = Solver(w, W0=W0, precision=a.precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv, n = False, 0
    chunk = 20000
    while not conv and n < a.ttr_max_steps:
        conv, n = s.step_until(a.ttr_target, min(chunk, a.ttr_max_steps - n))
        ri, ra, _ = s.residual()
        print(f"# step {n} r_inst {ri:.3e} r_avg {ra:.3e} {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    march = time.perf_counter() - t0
    elapsed = march + (ws_info["seconds"] if ws_info else 0.0)
    ri, ra, _ = s.residual()
    surf, cd = s.surface(1)
    start = ("learned warm start (coarse 40x30 UGKWP solve, BF16 MLP 32-256-256-256-32)" if a.warm_start
             else "uniform freestream")
    name = (f"cylinder O-grid 200x150, Ma 15, Kn {a.kn}, VHS omega 0.81, Pr 2/3, Tw/Tinf 0.2 diffuse, N_ref 400, "
            f"LTS CFL 0.8, {a.precision}, Philox seed 1" if a.workload == "cylinder" else
            f"flat plate 300x200, Ma 10, Kn 0.0169, VHS omega 0.74, Pr 1, Tw/Tinf 1 diffuse, N_ref 300, "
            f"LTS CFL 0.8, {a.precision}, Philox seed 1")
    out = {"metric": f"time-to-residual {a.ttr_target:g}", "value": elapsed if conv else None, "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "steps": int(n), "converged": bool(conv),
           "elapsed_s": elapsed, "march_s": march, "warm_start_s": ws_info["seconds"] if ws_info else 0.0,
           "ms_per_step": march / max(n, 1) * 1e3, "r_avg": ra, "r_inst": ri,
           "dtype": a.precision, "data": "synthetic",
           "config": {"workload": name,
                      "start": start, "dt_from": a.dt_source, "rule": "first n >= 100 with r_avg < target"},
           "wall": {"Cd_mean": cd, "Cp_max": float(np.max(surf[:, 3])), "CF_absmax": float(np.max(np.abs(surf[:, 4]))),
                    "CQ_max": float(np.max(surf[:, 5]))}}
    print(json.dumps(out))


def precision_study(a):
    """The Ma 10 flat plate (300 x 200, Kn 0.0169, N_ref 300) run for
    --study-steps steps from the freestream start: FP64 with seeds 1 and 2 and
    the mixed path with seeds 1 and 2.  Reports, for the cumulative-average
    wall C_p, C_F, C_Q (relative L2 norm over the 240 wall faces) and C_d, the
    mixed path's difference from FP64 seed 1 next to FP64's own difference
    between the seeds (the statistical spread)."""
    import numpy as np
    import torch
    from paper_2607_09552_amd import Solver
    runs = {}
    for prec, seed in (("f64", 1), ("f64", 2), ("mixed", 1), ("mixed", 2)):
        w = workloads.flat_plate(seed=seed)
        s = Solver(w, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(a.study_steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        surf, cd = s.surface(1)
        runs[(prec, seed)] = (surf[:, 3:6].copy(), cd, s.work() / t)
        print(f"# {prec} seed {seed}: {a.study_steps} steps in {t:.1f} s, C_d {cd:.5f}", file=sys.stderr, flush=True)
        s.close()
    ref, cd_ref, _ = runs[("f64", 1)]

    def rel(x):
        return [float(np.linalg.norm(x[:, q] - ref[:, q]) / np.linalg.norm(ref[:, q])) for q in range(3)]
    out = {"study": "mixed-precision wall-quantity error, flat plate",
           "config": {"workload": "flat plate 300x200, Ma 10, Kn 0.0169, VHS omega 0.74, Pr 1, Tw/Tinf 1 diffuse, "
                                  "N_ref 300, LTS CFL 0.8", "steps": a.study_steps,
                      "quantities": "cumulative averages over all steps from the freestream start"},
           "fp64_seed_spread": {"Cp_CF_CQ_rel_l2": rel(runs[("f64", 2)][0]),
                                "Cd_rel": abs(runs[("f64", 2)][1] - cd_ref) / abs(cd_ref)},
           "mixed_seed1_vs_fp64_seed1": {"Cp_CF_CQ_rel_l2": rel(runs[("mixed", 1)][0]),
                                         "Cd_rel": abs(runs[("mixed", 1)][1] - cd_ref) / abs(cd_ref)},
           "mixed_seed2_vs_fp64_seed1": {"Cp_CF_CQ_rel_l2": rel(runs[("mixed", 2)][0]),
                                         "Cd_rel": abs(runs[("mixed", 2)][1] - cd_ref) / abs(cd_ref)},
           "particle_updates_per_s": {f"{k[0]} seed {k[1]}": v[2] for k, v in runs.items()}}
    print(json.dumps(out))


def batch_bench(a):
    """Throughput of a batch of independent uneven cylinder cases in one
    context (one launch per kernel for all cases)."""
    import torch
    from paper_2607_09552_amd import Solver
    cases = workloads.cylinder_batch(a.batch)
    nc = int(sum(w["n_cells"] for w in cases))
    s = Solver.batch(cases, precision=a.precision)
    print(f"# batch of {a.batch} cases, {nc} cells; warmup {a.warmup} steps", file=sys.stderr, flush=True)
    s.step(a.warmup)
    s.profile(True, transport_only=True)
    torch.cuda.synchronize()
    w0 = s.work()
    t0 = time.perf_counter()
    s.step(a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_upd = s.work() - w0
    tr = s.profile_read()["transport"]
    s.profile(False)
    avg_ms = tr["ms"] / max(tr["launches"], 1)
    bytes_per_launch = TRANSPORT_BYTES[a.precision] * n_upd / max(tr["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    out = {"metric": "particle updates/s", "value": n_upd / elapsed, "unit": "particle updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": elapsed / a.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if a.precision == "f64" else "f32 particles, f64 cells", "data": "synthetic",
           "config": {"workload": f"batch of {a.batch} uneven cylinder cases (80x60 to 240x180 O-grids, Ma 5-20, "
                                  f"Kn 0.005-0.2, Tw/Tinf 0.1-0.5, N_ref 200, LTS), one batched solve",
                      "cases": a.batch, "cells": nc, "particles_per_step": n_upd / a.steps,
                      "cell_steps_per_s": nc * a.steps / elapsed},
           "roofline": {"bound": "hbm", "kernel": "transport", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "bytes_per_launch": bytes_per_launch, "avg_ms": avg_ms}}
    print(json.dumps(out))


MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_bench(a):
    """Matrix-core kernels of the warm-start network (32-256-256-256-32,
    GELU): inference over the 200x150 fine grid (30 016 rows) and training
    steps of 8192 rows, timed with HIP events on the stream they run on."""
    import numpy as np
    import torch
    from paper_2607_09552_amd import warmstart as ws
    mlp = ws.MLP(seed=0)
    wd = ws.WIDTHS
    macs = sum(i * o for i, o in zip(wd[:-1], wd[1:]))
    g = np.random.default_rng(0)

    def rand_bf16(rows, cols):
        x = g.standard_normal((rows, cols)).astype(np.float32)
        return torch.tensor((x.view(np.uint32) >> 16).astype(np.uint16).view(np.int16), device="cuda")

    def timed(fn, reps):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    M = ws.FINE[0] * ws.FINE[1] + (-ws.FINE[0] * ws.FINE[1]) % 32
    X = rand_bf16(M, wd[0])
    mlp.infer(X, M)
    fwd_ms = timed(lambda: mlp.infer(X, M), a.steps)
    fwd_tf = 2.0 * M * macs / (fwd_ms * 1e-3) / 1e12
    lay_ms = timed(lambda: mlp.forward(X, M), a.steps)
    Mt = 8192
    Xt, XTt = rand_bf16(Mt, wd[0]), rand_bf16(wd[0], Mt)
    T = torch.zeros((Mt, 4), dtype=torch.float32, device="cuda")
    tr_ms = timed(lambda: mlp.train_step(Xt, XTt, T, Mt, 1e-4, want_loss=False), a.steps)
    tr_tf = 6.0 * Mt * macs / (tr_ms * 1e-3) / 1e12
    out = {"metric": "warm-start network TFLOP/s (inference)", "value": fwd_tf, "unit": "TFLOP/s", "n_gpus": 1,
           "steps": a.steps, "warmup": 5, "ms_per_step": fwd_ms, "higher_is_better": True, "scaling": "strong",
           "vs_baseline": None, "dtype": "bf16 operands, f32 accumulation", "data": "synthetic",
           "config": {"workload": f"MLP {'-'.join(map(str, wd))} GELU, {M} rows (200x150 grid)",
                      "per_layer_ms": lay_ms, "per_layer_tflops": 2.0 * M * macs / (lay_ms * 1e-3) / 1e12,
                      "train_rows": Mt, "train_ms_per_step": tr_ms, "train_tflops": tr_tf},
           "roofline": {"bound": "mfma", "kernel": "k_mlp_fused", "achieved": fwd_tf,
                        "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": fwd_tf / MFMA_BF16_PEAK_TFLOPS,
                        "traffic": None, "flops_per_forward": 2.0 * M * macs}}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the throughput settles once the bow shock has formed (about 3000 steps
    # from the freestream start); the default times the developed flow
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 1000; 100 with --batch)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 3000; 200 with --batch)")
    ap.add_argument("--batch", type=int, default=0,
                    help="N > 0: N uneven cylinder cases (80x60 to 240x180, Ma 5-20, Kn 0.005-0.2, N_ref 200) "
                         "in one batched solve")
    ap.add_argument("--kn", type=float, default=0.01)
    ap.add_argument("--gts", action="store_true",
                    help="global time step (Eq. (34)) on the cylinder: per-step throughput at a step cap")
    ap.add_argument("--workload", choices=("cylinder", "plate"), default="cylinder",
                    help="plate: the Ma 10 flat plate (300x200, N_ref 300) instead of the cylinder")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--precision", choices=("f64", "mixed"), default="f64",
                    help="mixed: FP32 particle positions (cell-relative) and velocities, FP64 elsewhere")
    ap.add_argument("--precision-study", action="store_true",
                    help="flat plate: wall-quantity error of the mixed path against FP64 and FP64's seed spread")
    ap.add_argument("--study-steps", type=int, default=20000)
    ap.add_argument("--ttr", action="store_true",
                    help="time to residual: run from the freestream start until r_avg < --ttr-target")
    ap.add_argument("--ttr-target", type=float, default=1e-6)
    ap.add_argument("--ttr-max-steps", type=int, default=600000)
    ap.add_argument("--dt-source", choices=["initial", "freestream"], default="initial",
                    help="with --ttr: the state the local time steps are taken from (Eq. (33)): the initial "
                         "field (the paper) or the freestream, which gives a warm start the freestream start's steps")
    ap.add_argument("--mlp", action="store_true", help="matrix-core kernels of the warm-start network")
    ap.add_argument("--warm-start", action="store_true",
                    help="with --ttr: start from the learned warm start instead of the freestream")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = 100 if a.batch else 1000
    if a.warmup is None:
        a.warmup = 200 if a.batch else 3000
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU path is a "
              "domain-decomposition design, not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe()
        return
    from paper_2607_09552_amd import Solver

    if a.ttr:
        time_to_residual(a)
        return
    if a.mlp:
        a.steps = a.steps if a.steps != 1000 else 200
        mlp_bench(a)
        return
    if a.precision_study:
        precision_study(a)
        return
    if a.batch:
        batch_bench(a)
        return
    w = workload(a.kn, lts=0 if a.gts else 1) if a.workload == "cylinder" else workloads.flat_plate(seed=1)
    if a.gts and a.workload != "cylinder":
        print("--gts applies to the cylinder", file=sys.stderr)
        sys.exit(2)
    s = Solver(w, precision=a.precision)
    print(f"# warmup {a.warmup} steps", file=sys.stderr, flush=True)
    done = 0
    while done < a.warmup:
        k = min(500, a.warmup - done)
        s.step(k)
        done += k
        torch.cuda.synchronize()
        print(f"# warmup step {done}", file=sys.stderr, flush=True)
    # timed region: HIP events around the transport launches only (events
    # around every kernel would slow the step measurably)
    s.profile(True, transport_only=True)
    work0 = s.work()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_upd = s.work() - work0
    prof = s.profile_read()
    s.profile(False)
    print(f"# timed {a.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # per-kernel breakdown from a separate, untimed segment with events
    # around every kernel
    nb = min(a.steps, 50)
    s.profile(True)
    s.step(nb)
    breakdown = s.profile_read()
    s.profile(False)
    state = None
    if not a.no_cpu and a.precision == "f64":
        state = (s.fields(), s.particles(), a.warmup + a.steps + nb)
    tr = prof["transport"]
    avg_ms = tr["ms"] / max(tr["launches"], 1)
    # algorithmic bytes of one launch: the byte model per particle times the
    # particles one launch transports on average over the timed steps
    bytes_per_launch = TRANSPORT_BYTES[a.precision] * n_upd / max(tr["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # counters taken on the LTS cylinder at this precision
    mt = measured_traffic(a.precision) if (a.workload == "cylinder" and not a.gts) else None
    traffic = None
    if mt is not None and "transport" in mt["kernels"]:
        traffic = mt["kernels"]["transport"]["bytes_per_particle"] * n_upd / max(tr["launches"], 1)
    kern = {k: dict(ms_per_launch=round(v["ms"] / max(v["launches"], 1), 5),
                    GBs=round(v["bytes"] / max(v["ms"], 1e-12) * 1e-6, 1) if v["ms"] > 0 else None)
            for k, v in breakdown.items() if v["launches"] > 0}
    value = n_upd / elapsed
    # whole-step algorithmic bytes: every transported particle read and
    # written once, plus the cell and face data of a step
    rec2 = 120.0 if a.precision == "f64" else 80.0  # one record read and written
    step_bytes = rec2 * n_upd / a.steps + 400.0 * w["n_cells"]
    out = {
        "metric": "particle updates/s",
        "value": value,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "f64" else "f32 particles, f64 cells",
        "data": "synthetic",
        "config": {"workload": (f"cylinder O-grid 200x150, Ma 15, Kn {a.kn}, VHS omega 0.81, Pr 2/3, "
                                f"Tw/Tinf 0.2 diffuse, N_ref 400, {'GTS' if a.gts else 'LTS'} CFL 0.8, "
                                if a.workload == "cylinder" else
                                "flat plate 300x200, Ma 10, Kn 0.0169, VHS omega 0.74, Pr 1, Tw/Tinf 1 diffuse, "
                                "N_ref 300, LTS CFL 0.8, ")
                               + f"{'FP64' if a.precision == 'f64' else 'FP32 particle push'}, Philox seed 1",
                   "cells": int(w["n_cells"]),
                   "particles_per_step": n_upd / a.steps,
                   "cell_steps_per_s": w["n_cells"] * a.steps / elapsed},
        "roofline": {"bound": "hbm", "kernel": "transport", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_per_launch, "avg_ms": avg_ms},
        "step_roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                          "achieved": step_bytes / (elapsed / a.steps) / 1e9,
                          "frac": step_bytes / (elapsed / a.steps) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_step": step_bytes,
                          "model": f"{rec2:.0f} B per particle update (read + write one record) + 400 B per cell",
                          "measured_bytes_per_particle": None if mt is None else mt["step_bytes_per_particle"]},
        "kernels": kern,
        "kernels_note": f"per-kernel breakdown from {nb} further steps with events around every kernel",
        "residual_at_end": dict(zip(("r_inst", "r_avg", "step"), s.residual())),
    }
    if not a.no_cpu and a.precision == "f64":
        out["cpu_baseline"] = cpu_baseline(w, state, a.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
