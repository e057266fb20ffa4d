"""Host-side pieces of the run monitors (no GPU): the cell volumes the
per-cell particle share chi_i is divided by, for one case and for a batch."""
import numpy as np

import workloads
from paper_2607_09552_amd import Solver, metrics


def _holder(wl, cases):
    # a Solver shell with only its workloads: cell_volumes reads nothing else
    s = Solver.__new__(Solver)
    s.wl, s.cases = wl, cases
    return s


def test_cell_volumes_one_case_batch_and_1d():
    xs, ys = np.array([0.0, 0.5, 1.5, 3.0]), np.array([0.0, 0.25, 1.0])
    w = workloads.uniform2d(workloads.box2d(xs, ys))
    v = metrics.cell_volumes(_holder(w, None))
    expect = np.outer(np.diff(ys), np.diff(xs)).ravel()
    assert v.shape == (w["n_cells"],)
    assert np.allclose(np.sort(v), np.sort(expect), rtol=1e-14)
    assert np.isclose(v.sum(), 3.0, rtol=1e-14)
    vb = metrics.cell_volumes(_holder(w, [w, w]))
    assert np.array_equal(vb, np.concatenate([v, v]))
    s1 = workloads.shock1d(n_half=8)
    v1 = metrics.cell_volumes(_holder(s1, None))
    assert np.array_equal(v1, np.diff(np.asarray(s1["nodes"], dtype=np.float64)[:, 0]))
    assert np.all(v1 > 0)
