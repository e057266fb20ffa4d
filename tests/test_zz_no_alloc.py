"""ugkwp_step_noalloc (no device allocation, scratch in the library's static
device array) against ugkwp_step, through the C ABI (needs a gfx950 GPU)."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _everything(s):
    p = s.particles()
    Sm, Sp = s.tally()
    out = dict(W=s.fields(), Sm=Sm, Sp=Sp, counts=s.counts()[0], res=np.array(s.residual()), faces=s.face_flux(),
               **p)
    out.update({"h_" + k: v for k, v in s.history().items()})
    sf, cd = s.surface(1)
    out["surf"], out["cd"] = sf, cd
    return out, s.counts()[1], s.work()


def test_step_without_allocation_matches_ugkwp_step():
    """Two calls in a row on one device, the second on a smaller mesh (and
    with fewer steps): each gives bit for bit what ugkwp_step gives for the
    same case, so the shared scratch array holds nothing from the first
    call that the second sees."""
    from paper_2607_09552_amd import Solver
    cases = [(wl.cylinder(n_theta=40, n_r=30, n_ref=50, Pr=2.0 / 3.0), 30),
             (wl.cylinder(n_theta=24, n_r=18, n_ref=40, Pr=2.0 / 3.0, Ma=8.0, seed=4), 12)]
    for w, n in cases:
        ref = Solver(w, particle_capacity=400_000)
        ref.set_tuning(use_graph=0)
        ref.step(n)
        s = Solver(w, particle_capacity=400_000)
        s.step_noalloc(n)
        a, ia, wa = _everything(ref)
        b, ib, wb = _everything(s)
        assert ia == ib and wa == wb
        for k in a:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (w["n_cells"], k)
        # and the context steps on normally afterwards
        s.step(2)
        ref.step(2)
        assert np.array_equal(s.fields(), ref.fields())


def test_step_without_allocation_refuses_to_grow():
    from paper_2607_09552_amd import EOVERFLOW, Solver, UgkwpError
    s = Solver(wl.cylinder(n_theta=24, n_r=18, n_ref=40), particle_capacity=5000)
    with pytest.raises(UgkwpError) as e:
        s.step_noalloc(3)
    assert e.value.code == EOVERFLOW
    s.step(3)  # ugkwp_step grows the store; the context is intact
    s.step_noalloc(2)
