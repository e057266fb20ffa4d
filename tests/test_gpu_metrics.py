"""The JSON-lines run monitor (paper_2607_09552_amd.metrics) reads the
library's getters after each block of steps: its records must be those
getters' values (and be written one per block)."""
import json

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_run_logged_writes_one_record_per_block_from_the_getters(tmp_path):
    from paper_2607_09552_amd import Solver
    from paper_2607_09552_amd.metrics import cell_volumes, run_logged
    s = Solver(wl.cylinder(n_theta=40, n_r=30, n_ref=50, Pr=2.0 / 3.0))
    path = tmp_path / "run.jsonl"
    recs = run_logged(s, 50, 20, str(path))
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert lines == recs
    assert [r["step"] for r in lines] == [20, 40, 50]
    last = lines[-1]
    ri, ra, step = s.residual()
    assert (last["r_inst"], last["r_avg"], last["step"]) == (ri, ra, step)
    _, info = s.counts()
    assert last["particles"]["total"] == info["total"] and last["particles"]["new"] == info["new"]
    assert last["cd"]["last"] == s.surface(0)[1] and last["cd"]["ema"] == s.surface(2)[1]
    _, Sp = s.tally()
    chi = Sp[:, 0] / cell_volumes(s) / s.fields()[:, 0]
    assert last["chi"]["mean"] == float(chi.mean()) and 0.0 <= last["chi"]["min"] <= last["chi"]["max"]
    cp, cq = s.stagnation((-1.0, 0.0), mode=2)
    assert last["stagnation"] == {"Cp_ema": float(cp), "CQ_ema": float(cq)}
    # a wall-less 1D case logs no wall quantities
    s1 = Solver(wl.shock1d())
    r1 = run_logged(s1, 10, 10, str(tmp_path / "shock.jsonl"))
    assert len(r1) == 1 and "cd" not in r1[0] and np.isfinite(r1[0]["chi"]["mean"])
