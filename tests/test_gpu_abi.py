"""Error behaviour of the C ABI (include/ugkwp.h), called directly: every
documented argument check returns its code without touching the state, the
message of the last error names the fault, and the context keeps stepping
afterwards with the results it would have had."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

OK, EINVAL, EOVERFLOW, ESTATE = 0, -1, -4, -6


def _lib():
    from paper_2607_09552_amd import load_library
    return load_library()


def _msg(L, h):
    return L.ugkwp_last_error(h).decode()


def test_argument_checks_leave_the_context_usable():
    from paper_2607_09552_amd import Solver, _Tuning
    L = _lib()
    w = wl.shock1d(n_half=20, n_ref=40)
    s = Solver(w)
    ref = Solver(w)
    h = s.h
    i32, i64, d = C.c_int32(), C.c_int64(), C.c_double()
    # null context, negative counts, non-positive target, missing output
    assert L.ugkwp_step(None, 1) == EINVAL
    assert L.ugkwp_step(h, -1) == EINVAL
    assert L.ugkwp_step_until(h, 0.0, 10, C.byref(i32)) == EINVAL
    assert L.ugkwp_step_until(h, 1e-6, 10, None) == EINVAL
    assert L.ugkwp_get_fields(h, None) == EINVAL
    # a single context has exactly one case
    assert L.ugkwp_case_residual(h, 1, C.byref(d), C.byref(d)) == EINVAL
    assert L.ugkwp_case_range(h, -1, C.byref(i64), C.byref(i64), C.byref(i64), C.byref(i64)) == EINVAL
    # surface quantities need a step and a known averaging mode
    assert L.ugkwp_surface(h, 0, None, 0, C.byref(i64), C.byref(d)) == ESTATE
    assert "no step" in _msg(L, h)
    assert L.ugkwp_surface(h, 3, None, 0, C.byref(i64), C.byref(d)) == EINVAL
    # step counter bounds (the pid layout holds 2^20 steps)
    assert L.ugkwp_set_step(h, 1 << 20) == EINVAL
    assert L.ugkwp_set_step(h, -1) == EINVAL
    # tuning values out of range
    t = _Tuning(batch_steps=0, use_graph=0, transport_block=256, shakhov_lanes=4)
    assert L.ugkwp_set_tuning(h, C.byref(t)) == EINVAL
    t = _Tuning(batch_steps=8, use_graph=0, transport_block=100, shakhov_lanes=4)
    assert L.ugkwp_set_tuning(h, C.byref(t)) == EINVAL
    assert "out of range" in _msg(L, h)
    good = dict(batch_steps=8, use_graph=0, transport_block=256, shakhov_lanes=4, max_crossings=100,
                scatter_block=512, tally_block=256, flux_block=256)
    for knob in ("scatter_block", "tally_block", "flux_block"):
        for bad in (0, 32, 96, 1024) + ((512,) if knob != "scatter_block" else ()):
            t = _Tuning(**dict(good, **{knob: bad}))
            assert L.ugkwp_set_tuning(h, C.byref(t)) == EINVAL, (knob, bad)
    # none of it changed anything: both contexts give the same steps
    for c in (s, ref):
        c.step(5)
    assert np.array_equal(s.dt(), ref.dt())
    pg, pr = s.particles(), ref.particles()
    assert np.array_equal(pg["pid"], pr["pid"]) and np.array_equal(pg["cell"], pr["cell"])
    assert np.allclose(s.fields(), ref.fields(), rtol=0, atol=1e-12 * np.abs(ref.fields()).max())
    # a particle buffer too small for the set, and particles outside the mesh
    n = len(pg["pid"])
    assert n > 10
    buf = [np.zeros(4, dt) for dt in (np.uint64, np.int32, np.float64, np.float64, np.float64)]
    u = np.zeros(12)
    ptr = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    assert L.ugkwp_get_particles(h, 4, ptr(buf[0], C.c_uint64), ptr(buf[1], C.c_int32), ptr(buf[2], C.c_double),
                                 ptr(buf[3], C.c_double), ptr(u, C.c_double), None, C.byref(i64)) == EOVERFLOW
    assert "too small" in _msg(L, h)
    cell = np.array([w["n_cells"]], dtype=np.int32)
    one = np.ones(1)
    pid = np.array([1], dtype=np.uint64)
    assert L.ugkwp_set_particles(h, 1, ptr(pid, C.c_uint64), ptr(cell, C.c_int32), ptr(one, C.c_double),
                                 ptr(one, C.c_double), ptr(np.zeros(3), C.c_double), None) == EINVAL
    assert "out of range" in _msg(L, h)
    assert L.ugkwp_set_particles(h, -1, None, None, None, None, None, None) == EINVAL
    # too many steps for the pid layout: refused before any work
    assert L.ugkwp_set_step(h, (1 << 20) - 5) == OK
    assert L.ugkwp_step(h, 10) == EOVERFLOW
    assert L.ugkwp_set_step(h, 5) == OK
    # still usable, still in step with the reference
    for c in (s, ref):
        c.step(3)
    assert np.array_equal(s.particles()["pid"], ref.particles()["pid"])
    s.close()
    ref.close()


def test_init_checks():
    from paper_2607_09552_amd import Solver, UgkwpError
    L = _lib()
    w = wl.shock1d(n_half=10, n_ref=20)
    holder = Solver.__new__(Solver)
    holder._keep = []
    m, p, W = holder._marshal(w, None, None, 0, "f64")
    assert L.ugkwp_init(C.byref(m), C.byref(p), W.ctypes.data_as(C.POINTER(C.c_double)), None) == EINVAL
    # batches are 2D and share the gas
    with pytest.raises(UgkwpError, match="2D"):
        Solver.batch([w, w])
    box = wl.box2d(wl.graded(6, 1.2), wl.graded(4, 1.3, 0.5), wl.BC_SYMMETRY)
    a = wl.uniform2d(box, n_ref=20, seed=1)
    b = wl.uniform2d(box, n_ref=20, seed=2)
    b["gas"] = dict(b["gas"], Pr=2.0 / 3.0)
    with pytest.raises(UgkwpError, match="must equal case 0"):
        Solver.batch([a, b])
    # an unknown boundary type is refused
    c = dict(a)
    c["bface_type"] = a["bface_type"].copy()
    c["bface_type"][0] = 9
    with pytest.raises(UgkwpError, match="unknown type"):
        Solver(c)


def test_stream_copy_copies_and_checks_its_arguments():
    """ugkwp_stream_copy (the bandwidth reference): the copy equals its
    source for the default grid, a small grid (grid-stride loop and its
    tail) and one element per thread; misaligned, overlapping, empty or
    odd-sized requests are refused with EINVAL before anything runs."""
    import torch
    from paper_2607_09552_amd import load_library, stream_copy
    L = load_library()
    n = (1 << 20) + 3  # 16-byte elements: a ragged tail for every grid
    a = torch.arange(2 * n, dtype=torch.float64, device="cuda")
    for blocks in (0, 7, (n + 255) // 256):
        b = torch.full_like(a, -1.0)
        ms = stream_copy(b, a, reps=2, blocks=blocks)
        torch.cuda.synchronize()
        assert ms > 0 and torch.equal(a, b), blocks
    out = C.c_double()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    other = torch.empty_like(a)
    pa, pb = a.data_ptr(), other.data_ptr()
    EINVAL = -1
    assert L.ugkwp_stream_copy(C.c_void_p(pb), C.c_void_p(pa), 0, 1, 0, st, C.byref(out)) == EINVAL
    assert L.ugkwp_stream_copy(C.c_void_p(pb), C.c_void_p(pa), 24, 1, 0, st, C.byref(out)) == EINVAL
    assert L.ugkwp_stream_copy(C.c_void_p(pb + 8), C.c_void_p(pa), 32, 1, 0, st, C.byref(out)) == EINVAL
    assert L.ugkwp_stream_copy(C.c_void_p(pa + 16), C.c_void_p(pa), 64, 1, 0, st, C.byref(out)) == EINVAL
    assert L.ugkwp_stream_copy(C.c_void_p(pb), C.c_void_p(pa), 32, 0, 0, st, C.byref(out)) == EINVAL
    assert L.ugkwp_stream_copy(None, C.c_void_p(pa), 32, 1, 0, st, C.byref(out)) == EINVAL
