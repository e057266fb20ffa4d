"""Launch-tuning sweep on the GPU (gfx950): steps per host synchronization,
graph replay, the block sizes of the transport, the re-sort's scatter, the
per-cell tally and the face fluxes, and the lanes per particle of the
Shakhov sampler's first phase (ugkwp_set_tuning; results do not depend on
them).

The flow keeps evolving while it is measured, so candidates are interleaved:
each round times every candidate for a few steps in turn, and the median
over rounds of each candidate's ms per particle update decides.  Candidates
are varied one knob at a time from the current best, and a knob keeps its
current value unless another beats it by more than NOISE (run-to-run spread
of the medians): a setting that only won within the noise can cost in ways
the timing does not show (a tally block of one wavefront, for instance,
spreads neighbouring cells over the device's L2 caches and fetches more).  The result is written
to tuning_gfx950.json beside this file, keyed by workload name; Solver
applies it when a workload of that name is built.

    python -m paper_2607_09552_amd.autotune [--workload cylinder|flat_plate] [--rounds 7]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_FILE = os.path.join(HERE, "tuning_gfx950.json")

SPACE = {
    "batch_steps": [8, 16, 32, 64],
    "use_graph": [0, 1],
    "transport_block": [64, 128, 256],
    "shakhov_lanes": [1, 2, 4, 8, 16],
    "scatter_block": [128, 256, 512],
    "tally_block": [64, 128, 256],
    "flux_block": [64, 128, 256],
}


NOISE = 0.005


def load_tuning(name):
    """Recorded best tuning for a workload name, or None."""
    try:
        with open(TUNING_FILE) as f:
            return json.load(f).get(name, {}).get("best")
    except (OSError, ValueError):
        return None


def _gpu_sync():
    import torch
    torch.cuda.synchronize()


def _time(solver, steps, clock, sync):
    sync()
    w0 = solver.work()
    t0 = clock()
    solver.step(steps)
    sync()
    return (clock() - t0) / max(solver.work() - w0, 1)


def sweep(solver, rounds=7, steps=64, log=print, clock=time.perf_counter, sync=_gpu_sync):
    best = solver.tuning()
    table = {}
    for knob, values in SPACE.items():
        cands = [dict(best, **{knob: v}) for v in values]
        times = [[] for _ in cands]
        for _ in range(rounds):
            for k, cfg in enumerate(cands):
                solver.set_tuning(**cfg)
                solver.step(2 * cfg["batch_steps"])  # settle (graph capture)
                times[k].append(_time(solver, steps, clock, sync))
        med = [sorted(t)[len(t) // 2] for t in times]
        k = min(range(len(cands)), key=lambda i: med[i])
        cur = values.index(best[knob]) if best[knob] in values else None
        if cur is not None and med[k] > med[cur] * (1.0 - NOISE):
            k = cur
        for cfg, m in zip(cands, med):
            table[json.dumps(cfg, sort_keys=True)] = m
        log(f"# {knob}: " + ", ".join(f"{c[knob]}: {m * 1e12:.2f} ps/update" for c, m in zip(cands, med)))
        best = cands[k]
    solver.set_tuning(**best)
    return best, table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("cylinder", "flat_plate"), default="cylinder")
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--rounds", type=int, default=7)
    ap.add_argument("--steps", type=int, default=64)
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    if not torch.cuda.is_available():
        sys.exit("no GPU visible")
    torch.cuda.set_device(0)  # initialize torch's device before the library's
    import workloads
    from paper_2607_09552_amd import Solver
    if a.workload == "cylinder":
        w = workloads.cylinder()
    else:
        w = workloads.flat_plate()
    s = Solver(w, tuned=False)
    s.step(a.warmup)
    best, table = sweep(s, a.rounds, a.steps, log=lambda m: print(m, file=sys.stderr, flush=True))
    try:
        with open(TUNING_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[w["name"]] = {"best": best, "seconds_per_update": table,
                       "command": f"python -m paper_2607_09552_amd.autotune --workload {a.workload} "
                                  f"--warmup {a.warmup} --rounds {a.rounds} --steps {a.steps}"}
    with open(TUNING_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({"workload": w["name"], "best": best}))


if __name__ == "__main__":
    main()
