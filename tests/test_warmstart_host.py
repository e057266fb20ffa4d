"""Host-side logic of the warm start (no GPU): the coarse grid is the fine
grid's every fifth node, so interpolation in cell-index space is
interpolation between coincident geometry; case draws and case records."""
import math

import numpy as np

from paper_2607_09552_amd import warmstart as ws


def test_coarse_nodes_are_every_fifth_fine_node():
    fine = ws.fine_case(10.0, 0.02, 0.3, n_ref=1)
    coarse = ws.coarse_case(10.0, 0.02, 0.3)
    nt, nr = ws.FINE
    ct, cr = ws.COARSE
    F = fine["nodes"].reshape(nr + 1, nt, 2)
    Cn = coarse["nodes"].reshape(cr + 1, ct, 2)
    sub = F[:: nr // cr, :: nt // ct]
    assert sub.shape == Cn.shape
    assert np.allclose(Cn, sub, rtol=0, atol=1e-12 * 15.0)
    # same wall temperature, free stream and gas
    assert np.array_equal(coarse["bface_data"][:ct, 0], np.full(ct, 0.3))
    assert coarse["ref"] == fine["ref"] and coarse["gas"] == fine["gas"]


def test_draws_cover_the_ranges_and_repeat():
    d = ws.draws(2000, 3)
    assert np.array_equal(d, ws.draws(2000, 3))
    assert not np.array_equal(d[:16], ws.draws(16, 4))
    for k, (lo, hi) in enumerate((ws.MA_RANGE, ws.KN_RANGE, ws.TW_RANGE)):
        assert lo <= d[:, k].min() and d[:, k].max() < hi
    # Kn is log-uniform: the median sits at the geometric mean
    assert abs(math.log(np.median(d[:, 1])) - 0.5 * math.log(0.005 * 0.2)) < 0.15


def test_case_record_matches_the_workload():
    w = ws.fine_case(13.0, 0.05, 0.2, n_ref=1)
    a, b = ws.ws_case(w, 13.0, 0.05, 0.2), ws.cylinder_ws_case(13.0, 0.05, 0.2)
    for f, _ in a._fields_:
        assert abs(getattr(a, f) - getattr(b, f)) <= 1e-12 * max(1.0, abs(getattr(a, f))), f
