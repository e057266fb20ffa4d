"""Step-block metrics as JSON lines: the run monitors of the paper's Sec. V
(residuals, the drag coefficient's history, the EMA of the stagnation
pressure and heat flux, the share of the mass carried by particles) and the
step's particle counts, read through the library's getters after every
block of steps.

Each line: {"step", "r_inst", "r_avg", "particles": {total, new, removed,
exited, guard}, "shakhov_fallbacks", "chi": {mean, min, max},
"cd": {last, mean, ema}, "stagnation": {Cp_ema, CQ_ema}} (the last two when
the case has walls).  chi_i = rho^{p,+}_i / rho_i is the density carried by
the particles that ended the last step in cell i (W^{p,+}, Eq. (30)) over
the cell's density after the update; its statistics are over the cells.
A host-side diagnostic: nothing here is part of the step.

    from paper_2607_09552_amd.metrics import run_logged
    run_logged(solver, n_steps=20000, every=1000, path="run.jsonl")
"""
from __future__ import annotations

import json

import numpy as np


def _volumes(w):
    if w["dim"] == 1:
        return np.diff(np.asarray(w["nodes"], dtype=np.float64)[:, 0])
    cp, cn, xy = w["cell_ptr"], w["cell_nodes"], np.asarray(w["nodes"], dtype=np.float64)
    p = [xy[cn[cp[i]:cp[i + 1]]] for i in range(w["n_cells"])]
    return np.array([0.5 * np.sum(q[:, 0] * np.roll(q[:, 1], -1) - np.roll(q[:, 0], -1) * q[:, 1]) for q in p])


def cell_volumes(solver):
    """Cell volumes (areas in 2D, lengths in 1D) from the solver's workload(s),
    in the context's cell order (a batch's cases one after another)."""
    if solver.cases is not None:
        return np.concatenate([_volumes(w) for w in solver.cases])
    return _volumes(solver.wl)


def record(solver, vol=None, stagnation_point=(-1.0, 0.0)):
    """One metrics record of the solver's last committed step."""
    ri, ra, step = solver.residual()
    _, info = solver.counts()
    rec = {"step": int(step), "r_inst": ri, "r_avg": ra,
           "particles": {k: int(info[k]) for k in ("total", "new", "removed", "exited", "guard")},
           "shakhov_fallbacks": int(solver.shakhov_fallbacks())}
    if step > 0:
        vol = cell_volumes(solver) if vol is None else vol
        _, Sp = solver.tally()
        rho = solver.fields()[:, 0]
        chi = Sp[:, 0] / vol / rho
        rec["chi"] = {"mean": float(chi.mean()), "min": float(chi.min()), "max": float(chi.max())}
        if solver.ncase == 1 and solver.n_wall() > 0:
            cd = [solver.surface(m)[1] for m in (0, 1, 2)]
            rec["cd"] = {"last": cd[0], "mean": cd[1], "ema": cd[2]}
            cp, cq = solver.stagnation(stagnation_point, mode=2)
            rec["stagnation"] = {"Cp_ema": float(cp), "CQ_ema": float(cq)}
    return rec


def run_logged(solver, n_steps, every, path, stagnation_point=(-1.0, 0.0)):
    """Advances the solver n_steps in blocks of `every` steps and appends one
    record per block to the JSON-lines file `path`; returns the records."""
    vol = cell_volumes(solver)
    out = []
    done = 0
    with open(path, "a") as f:
        while done < n_steps:
            k = min(every, n_steps - done)
            solver.step(k)
            done += k
            rec = record(solver, vol, stagnation_point)
            f.write(json.dumps(rec) + "\n")
            f.flush()
            out.append(rec)
    return out
