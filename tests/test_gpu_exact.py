"""Reproducibility, checkpoints, failure handling and stage-level parity of the
HIP path (needs a gfx950 GPU; every call goes through the C ABI).

- reproducibility: the particle tallies of Eqs. (24), (29)-(30), the wall
  impulses and the residual sums are exact fixed-point sums, so two runs
  from the same seed agree bit for bit in fields, particles, tallies, wall
  quantities and residuals, whatever order the GPU's atomics take;
- checkpoints: N steps, save, load into a fresh context, N steps equals 2N
  uninterrupted steps bit for bit (FP64 and mixed precision);
- failures are not committed: a step that fails leaves fields, particles,
  tallies, averages and the step counter as they were, and the context
  steps on as if the failed call had not happened;
- stage-level parity with the oracle from a common state, each quantity on
  its own scale: face fluxes F_j s_j on every kind of face, the field change
  dW = W^{n+1} - W^n, the tallies, wall quantities and residuals.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _solver(w, **kw):
    from paper_2607_09552_amd import Solver
    return Solver(w, **kw)


def _state(s):
    """Everything a run exposes after a step, for bit-for-bit comparisons."""
    p = s.particles()
    Sm, Sp = s.tally()
    out = dict(W=s.fields(), tally_m=Sm, tally_p=Sp, counts=s.counts()[0], info=s.counts()[1],
               res=np.array(s.residual()), faces=s.face_flux(), fallbacks=s.shakhov_fallbacks(), **p)
    for k, v in s.history().items():
        out["h_" + k] = v
    if s.n_wall():
        for mode in (0, 1, 2):
            sf, cd = s.surface(mode)
            out[f"surf{mode}"] = sf
            out[f"cd{mode}"] = cd
    return out


def _assert_identical(a, b, tag):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, dict):
            assert x == y, f"{tag}: {k} {x} vs {y}"
        else:
            assert np.array_equal(np.asarray(x), np.asarray(y)), f"{tag}: {k} differs"


def _cylinder(**kw):
    return wl.cylinder(n_theta=40, n_r=30, n_ref=50, Pr=2.0 / 3.0, **kw)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_same_seed_runs_are_bit_identical(precision):
    """Two independent runs of the 40 x 30 Ma 15 cylinder (Shakhov, Pr 2/3:
    raw-moment tallies too) over 200 steps, one with graph replays and one
    with eager launches and other block shapes: every field, particle,
    tally, face flux, wall quantity and residual identical (FP64 and the
    mixed-precision store)."""
    w = _cylinder()
    a = _solver(w, precision=precision)
    b = _solver(w, precision=precision)
    a.set_tuning(use_graph=1, batch_steps=16)
    b.set_tuning(use_graph=0, batch_steps=7, transport_block=128, shakhov_lanes=8, scatter_block=64,
                 tally_block=128, flux_block=64)
    for n in (1, 50, 200):
        a.step(n - a.residual()[2])
        b.step(n - b.residual()[2])
        _assert_identical(_state(a), _state(b), f"step {n}")


def test_side_stream_matches_the_serial_order():
    """The face fluxes on the side stream beside the re-sort (graph replays)
    and in order on the library stream (per-kernel timing on, eager
    launches): identical states after 60 steps."""
    w = _cylinder()
    a = _solver(w)
    b = _solver(w)
    a.set_tuning(use_graph=1, batch_steps=16)
    b.profile(True)
    for n in (1, 60):
        a.step(n - a.residual()[2])
        b.step(n - b.residual()[2])
        _assert_identical(_state(a), _state(b), f"step {n}")
    b.profile(False)


def test_batch_is_reproducible():
    """The same for a batch of uneven cases (per-case residual and drag sums)."""
    from paper_2607_09552_amd import Solver
    cases = [_cylinder(Ma=10.0, seed=3), wl.cylinder(n_theta=24, n_r=18, n_ref=50, Pr=2.0 / 3.0, Ma=6.0, seed=9)]
    a, b = Solver.batch(cases), Solver.batch(cases)
    b.set_tuning(use_graph=0, batch_steps=5)
    a.step(60)
    b.step(60)
    _assert_identical(_state(a), _state(b), "batch")
    for k in range(2):
        assert a.case_residual(k) == b.case_residual(k)
        sa, ca = a.case_surface(k, 1)
        sb, cb = b.case_surface(k, 1)
        assert np.array_equal(sa, sb) and ca == cb


@pytest.mark.parametrize("which", ["shock", "cylinder", "cylinder_mixed"])
def test_checkpoint_round_trip_is_bit_exact(which, tmp_path):
    """N steps, ugkwp_save, ugkwp_load into a fresh context, N more steps:
    identical to 2N uninterrupted steps (averages, surfaces, residual
    history and the work counter included)."""
    precision = "mixed" if which == "cylinder_mixed" else "f64"
    w = wl.shock1d(n_ref=100) if which == "shock" else _cylinder()
    N = 40 if which == "shock" else 25
    ref = _solver(w, precision=precision)
    ref.step(2 * N)
    a = _solver(w, precision=precision)
    a.step(N)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    assert os.path.getsize(path) > 0 and not os.path.exists(path + ".tmp")
    b = _solver(w, precision=precision)
    b.load(path)
    committed = lambda s: {k: v for k, v in _state(s).items() if k not in ("faces", "tally_m", "tally_p")}
    _assert_identical(committed(a), committed(b), "after load")
    assert a.work() == b.work()
    b.step(N)
    _assert_identical(_state(ref), _state(b), "continued")
    assert ref.work() == b.work()


def test_checkpoint_rejects_a_mismatched_context(tmp_path):
    from paper_2607_09552_amd import EINVAL, EIO, UgkwpError
    a = _solver(_cylinder())
    a.step(3)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    other = _solver(wl.cylinder(n_theta=24, n_r=18, n_ref=40))
    with pytest.raises(UgkwpError) as e:
        other.load(path)
    assert e.value.code == EINVAL
    with pytest.raises(UgkwpError) as e:
        other.load(str(tmp_path / "missing.bin"))
    assert e.value.code == EIO
    other.step(2)  # still usable


def _snapshot(s):
    st = _state(s)
    st.pop("faces")
    return st


def test_failed_steps_are_not_committed():
    """(1) An invalid field loaded through ugkwp_set_fields: the step fails
    (ENUMERIC) before anything is modified.  (2) A runaway track forced from
    the host (at most one face crossing per particle and step): the step
    fails after transport has run, and still nothing of it is committed.  In
    both cases the state afterwards is the last committed one, and the
    context, given back a valid state or its tuning, continues exactly like
    a context that never failed."""
    from paper_2607_09552_amd import ENUMERIC, UgkwpError
    w = _cylinder()
    ref = _solver(w)
    s = _solver(w)
    for x in (ref, s):
        x.step(12)
    before = _snapshot(s)
    W = s.fields()
    bad = W.copy()
    bad[7, 3] = -1.0  # negative energy: not a Maxwellian (the density is kept)
    s.set_fields(bad)
    with pytest.raises(UgkwpError) as e:
        s.step(3)
    assert e.value.code == ENUMERIC
    _assert_identical(_snapshot(s), dict(before, W=bad), "after the invalid state")
    s.set_fields(W)
    _assert_identical(_snapshot(s), before, "valid state restored")
    # (2) runaway
    s.set_tuning(max_crossings=1)
    with pytest.raises(UgkwpError) as e:
        s.step(4)
    assert e.value.code == ENUMERIC and "runaway" in str(e.value)
    _assert_identical(_snapshot(s), before, "after the runaway")
    s.set_tuning(max_crossings=10000)
    s.step(10)
    ref.step(10)
    _assert_identical(_state(s), _state(ref), "continued after the failures")


# ---------------------------------------------------------------------------
# stage-level parity from a common state
# ---------------------------------------------------------------------------

def _vol(w):
    if w["dim"] == 1:
        return np.diff(w["nodes"][:, 0])
    cp, cn, xy = w["cell_ptr"], w["cell_nodes"], w["nodes"]
    vol = np.zeros(w["n_cells"])
    for i in range(w["n_cells"]):
        p = xy[cn[cp[i]:cp[i + 1]]]
        vol[i] = 0.5 * np.sum(p[:, 0] * np.roll(p[:, 1], -1) - np.roll(p[:, 0], -1) * p[:, 1])
    return vol


def _scaled_err(a, b, scale=None):
    """max |a - b| per column over that column's max |b| (or `scale`)."""
    s = np.abs(b).max(axis=0) if scale is None else scale
    s = np.where(s == 0, 1.0, s)
    return float(np.max(np.abs(a - b).max(axis=0) / s))


def _tally_err(a, b):
    """A tally S = sum m Psi on its own scale: max |S_rho|, max |S_E| and,
    for momentum, max sqrt(2 |S_rho| |S_E|), the bound of sum m |u|."""
    nw = b.shape[1]
    scale = np.abs(b).max(axis=0)
    scale[1:nw - 1] = np.sqrt(2.0 * np.abs(b[:, 0]) * np.abs(b[:, nw - 1])).max()
    return _scaled_err(a, b, scale)


def common_state_stage_parity(w, n, tag):
    """Run the GPU to step n, load fields, particles, step counter and the
    averaging state into a fresh GPU context and the oracle, take one step
    on both, and compare every stage on its own scale."""
    free = _solver(w)
    free.step(n)
    W, p, h = free.fields(), free.particles(), free.history()
    g = _solver(w)
    r = oracle.Oracle(w)
    for s in (g, r):
        s.set_fields(W)
        if len(p["pid"]):
            s.set_particles(p["pid"], p["cell"], p["m"], p["x"], p["u"], p["ei"])
        s.set_step(n)
    g.set_history(h)
    r.set_history(dict(rho_prev=h["rho_prev"], rho_sum=h["rho_sum"], rho_mean_prev=h["rho_mean_prev"],
                       wlast=h["wlast"], wsum=h["wsum"], wema=h["wema"], cd=h["scal"][2:5]))
    g.step(1)
    r.step(1)
    pg, pr = g.particles(), r.particles()
    assert np.array_equal(pg["pid"], pr["pid"]) and np.array_equal(pg["cell"], pr["cell"]), tag
    assert np.array_equal(g.counts()[0], r.counts()[0]), tag
    assert g.counts()[1] == r.counts()[1], tag
    assert g.shakhov_fallbacks() == r.n_capped(), tag
    errs = {}
    Fg, Fr = g.face_flux(), r.face_flux()
    errs["face flux"] = _scaled_err(Fg, Fr)
    Wg, Wr = g.fields(), r.fields()
    errs["dW"] = _scaled_err(Wg - W, Wr - W)
    Smg, Spg = g.tally()
    Smr, Spr = r.tally()
    errs["W^{p,-}"] = _tally_err(Smg, Smr)
    errs["W^{p,+}"] = _tally_err(Spg, Spr)
    ig, ag, _ = g.residual()
    ir, ar, _ = r.residual()
    errs["r_inst"] = abs(ig - ir) / ir
    errs["r_avg"] = abs(ag - ar) / ar if ar > 0 else abs(ag)
    if g.n_wall():
        for mode in (0, 1, 2):
            sg, cdg = g.surface(mode)
            sr, cdr = r.surface(mode)
            errs[f"surface {mode}"] = _scaled_err(sg[:, 3:], sr[:, 3:])
            errs[f"C_d {mode}"] = abs(cdg - cdr) / abs(cdr)
    bad = {k: v for k, v in errs.items() if not v <= TOL}
    assert not bad, f"{tag}: {bad} (all: {errs})"
    return errs


def test_stage_parity_flat_plate_every_face_type():
    """Ma 10 flat plate at full size (300 x 200): inflow and top far-field
    faces, the outflow face, the symmetry plane and the diffuse plate, one
    step from the state after 300 steps; then the same with the plate a
    Maxwell wall (alpha = 0.85) on a coarser plate."""
    common_state_stage_parity(wl.flat_plate(), 300, "plate")
    m = wl.with_maxwell_walls(wl.flat_plate(n_up=15, n_plate=60, n_y=50, n_ref=80), 0.85)
    common_state_stage_parity(m, 60, "Maxwell plate")


def test_stage_parity_cylinder_full_size():
    """The benchmark cylinder (200 x 150, Ma 15, Kn 0.01, Shakhov) one step
    from the state after 400 steps: bow shock forming, a near-vacuum wake."""
    import bench
    common_state_stage_parity(bench.workload(), 400, "cylinder")


def test_stage_parity_shock_and_gts():
    common_state_stage_parity(wl.shock1d(), 700, "shock")
    common_state_stage_parity(dict(wl.shock1d(), lts=0), 60, "shock, GTS")
