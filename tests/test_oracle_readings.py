"""Pins of the oracle's readings where the paper is silent.

- exactly rounded sums (the tallies of Eqs. (24), (29)-(30)) against exact
  rational arithmetic;
- MUSCL/van Leer reconstruction and the central equilibrium slope: exact on
  linear fields over graded 1D and 2D meshes, the limiter's closed form, the
  first-order fallbacks;
- the vacuum guard: each branch against its definition, and firing in a
  rarefaction that empties a cell;
- the Shakhov sampler's 64-attempt fallback: the first draw inside the cut.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl


# ---------------------------------------------------------------------------
# exact sums
# ---------------------------------------------------------------------------

def _exact(xs):
    return float(sum((Fraction(x) for x in xs), Fraction(0)))


def test_exact_sum_is_the_correctly_rounded_sum():
    """The oracle's sum of doubles equals the exact rational sum rounded to
    nearest (ties to even): random sets over wide exponent ranges, massive
    cancellation, and constructed half-way ties (a dropped partial, a wrong
    tie rule or a plain running sum fails these)."""
    rng = np.random.default_rng(11)
    cases = []
    for n in (1, 2, 3, 10, 100, 1000):
        cases.append(rng.normal(size=n))
        cases.append(rng.normal(size=n) * np.exp2(rng.integers(-60, 60, size=n)))
        x = rng.normal(size=n) * np.exp2(rng.integers(-30, 30, size=n))
        cases.append(np.concatenate([x, -x[::-1], rng.normal(size=3) * 1e-20]))
    # half-way cases: 1 + 2^-53 ties to 1, 1 + 3 * 2^-53 ties up, a tiny tail
    # below decides the tie's direction
    u = 2.0 ** -53
    cases += [np.array([1.0, u]), np.array([1.0, 3 * u]), np.array([1.0, u, u * u]),
              np.array([1.0, u, -u * u]), np.array([1.0 + 2 * u, u]), np.array([-1.0, -u, -(u * u)]),
              np.array([1e300, 1e300, -1e300]), np.array([0.1] * 10), np.array([])]
    for x in cases:
        got = oracle.exact_sum(x)
        assert got == _exact(x), (x[:5], got, _exact(x))
        assert oracle.exact_sum(x[::-1]) == got
        assert oracle.exact_sum(rng.permutation(x)) == got


# ---------------------------------------------------------------------------
# reconstruction and the equilibrium slope
# ---------------------------------------------------------------------------

def _state(p):
    """A valid face-frame state (rho, rho U, rho V, rho E) for K = 1."""
    return np.array(p, dtype=np.float64)


def test_reconstruction_exact_on_linear_profiles():
    """A field linear along the face normal is reconstructed exactly at the
    face (xi = 0) with its slope, whatever the (graded) centroid spacing:
    the one-sided differences are weighted by the centroid distances and
    the van Leer limiter of two equal slopes is that slope."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = _state([rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(8, 12)])
        b = rng.normal(size=4) * 0.05
        xself = -rng.uniform(0.01, 2.0)
        xfar = xself - rng.uniform(0.01, 3.0)
        xother = rng.uniform(0.01, 2.0)
        W = lambda x: a + b * x
        out, slope = oracle.reconstruct(W(xfar), xfar, W(xself), xself, W(xother), xother)
        assert np.allclose(out, a, rtol=0, atol=1e-14 * np.abs(a).max())
        assert np.allclose(slope, b, rtol=1e-12, atol=1e-16)


def test_van_leer_limiter_closed_form_and_fallbacks():
    """Unequal one-sided slopes d1, d2 of one sign give 2 d1 d2 / (d1 + d2)
    (not the mean, not minmod); opposite signs (an extremum) give 0; a
    limited face value that is not a valid Maxwellian, or a missing far
    neighbour, gives the first-order value."""
    xfar, xself, xother = -3.0, -1.0, 0.5
    Wself = _state([1.0, 0.1, 0.0, 10.0])
    d1 = np.array([0.2, -0.1, 0.05, 0.3])
    d2 = np.array([0.05, -0.4, 0.2, 0.1])
    Wfar = Wself - d1 * (xself - xfar)
    Wother = Wself + d2 * (xother - xself)
    out, slope = oracle.reconstruct(Wfar, xfar, Wself, xself, Wother, xother)
    vl = 2 * d1 * d2 / (d1 + d2)
    assert np.allclose(slope, vl, rtol=1e-13)
    assert np.allclose(out, Wself - vl * xself, rtol=1e-13)
    # extremum in the momentum component only
    Wother2 = Wother.copy()
    Wother2[1] = Wself[1] + 0.3 * (xother - xself)
    out, slope = oracle.reconstruct(Wfar, xfar, Wself, xself, Wother2, xother)
    assert slope[1] == 0.0 and out[1] == Wself[1] and slope[0] != 0.0
    # valid neighbours whose limited extrapolation overshoots to a negative
    # face density (the face lies farther from the cell centroid than half
    # the distance to the other centroid): first order everywhere
    Wb = _state([0.2, 0.0, 0.0, 1.0])
    Wf = _state([0.2 + 5.0 * 4.0, 0.0, 0.0, 1.0])
    Wo = _state([0.2 - 0.075 * 2.5, 0.0, 0.0, 1.0])
    out, slope = oracle.reconstruct(Wf, -6.0, Wb, -2.0, Wo, 0.5)
    assert np.array_equal(out, Wb) and np.array_equal(slope, np.zeros(4))
    out, slope = oracle.reconstruct(None, 0.0, Wself, xself, Wother, xother)
    assert np.array_equal(out, Wself) and np.array_equal(slope, np.zeros(4))


def _centroids(m):
    if m["dim"] == 1:
        x = m["nodes"][:, 0]
        return np.stack([0.5 * (x[:-1] + x[1:]), np.zeros(len(x) - 1)], axis=1)
    nodes = m["nodes"]
    cp, cn = m["cell_ptr"], m["cell_nodes"]
    out = []
    for i in range(m["n_cells"]):
        p = nodes[cn[cp[i]:cp[i + 1]]]
        x, y = p[:, 0], p[:, 1]
        xn, yn = np.roll(x, -1), np.roll(y, -1)
        cr = x * yn - xn * y
        A = 0.5 * cr.sum()
        out.append([((x + xn) * cr).sum() / (6 * A), ((y + yn) * cr).sum() / (6 * A)])
    return np.array(out)


def _frame(W, n, dim):
    if dim == 1:
        return np.array([W[0], W[1] * n[0], 0.0, W[2]])
    return np.array([W[0], W[1] * n[0] + W[2] * n[1], W[2] * n[0] - W[1] * n[1], W[3]])


@pytest.mark.parametrize("dim", [1, 2])
def test_face_values_exact_on_linear_fields_over_graded_meshes(dim):
    """Every interior face of a graded mesh: for W linear in space, both
    sides reconstruct the field's value at the face midpoint and its normal
    slope, and the equilibrium slope (central difference of the cell
    averages along n) is that normal slope too; sides without a cell across
    their opposite face are first order.  A slope off by a factor, an
    unweighted difference or a transposed side fails it."""
    if dim == 1:
        m = wl.uniform1d(np.concatenate([-wl.graded(5, 1.3)[::-1], wl.graded(6, 1.2)[1:]]))
    else:
        m = wl.uniform2d(wl.box2d(wl.graded(6, 1.25), wl.graded(5, 1.4, 0.5)))
    cen = _centroids(m)
    nw = dim + 2
    a = np.array([1.0, 0.2, -0.1, 12.0])[:nw] if dim == 2 else np.array([1.0, 0.2, 12.0])
    Gx = np.array([0.02, -0.01, 0.015, 0.1])[:nw] if dim == 2 else np.array([0.02, -0.01, 0.1])
    Gy = np.array([-0.03, 0.02, 0.01, -0.2])[:nw] if dim == 2 else np.zeros(3)
    W = a + cen[:, :1] * Gx + cen[:, 1:] * Gy
    o = oracle.Oracle(m)
    o.set_fields(W)
    checked = 0
    for fi in range(o.nf):
        g = o.face_geom(fi)
        if g["R"] < 0:
            continue
        n = g["n"]
        Wface = a + g["mid"][0] * Gx + g["mid"][1] * Gy
        grad_n = Gx * n[0] + Gy * n[1]
        ref_face = _frame(Wface, n, dim)
        ref_slope = _frame(grad_n, n, dim) - (_frame(np.zeros(nw), n, dim))
        WLf, WRf, sl, sr, dW0 = o.face_values(fi)
        scale = np.abs(ref_face).max()
        assert np.allclose(dW0, ref_slope, rtol=1e-11, atol=1e-13)
        for Wf, s, far, cell in ((WLf, sl, g["LL"], g["L"]), (WRf, sr, g["RR"], g["R"])):
            if far >= 0:
                assert np.allclose(Wf, ref_face, rtol=0, atol=1e-13 * scale), (fi, Wf, ref_face)
                assert np.allclose(s, ref_slope, rtol=1e-11, atol=1e-13)
                checked += 1
            else:
                assert np.array_equal(Wf, _frame(W[cell], n, dim)) and not s.any()
    assert checked >= (8 if dim == 1 else 40)


# ---------------------------------------------------------------------------
# vacuum guard
# ---------------------------------------------------------------------------

def test_vacuum_guard_branches():
    """A valid updated state is kept; an invalid one takes the particles'
    content Sp / Omega when that is a valid state, else the floor state
    (rho = 1e-12 rho_inf at rest, temperature T_inf)."""
    m = wl.uniform2d(wl.box2d(wl.graded(2, 1.0), wl.graded(2, 1.0)), rho=2.0, T=3.0)
    o = oracle.Oracle(m)
    vol = 0.37
    ok_state = wl.conservative(1.0, 0.3, -0.2, 1.5, 2)
    fired, Wn = o.vacuum_guard(np.zeros(4), vol, ok_state)
    assert not fired and np.array_equal(Wn, ok_state)
    bad = np.array([0.5, 0.1, 0.0, -1e-3])              # negative internal energy
    Sp = wl.conservative(0.2, 1.0, 0.5, 0.7, 2) * vol    # particles' content times Omega
    fired, Wn = o.vacuum_guard(Sp, vol, bad)
    assert fired and np.array_equal(Wn, Sp / vol)
    for Sp_bad in (np.zeros(4), np.array([0.1, 0.5, 0.0, 0.0]) * vol, np.array([-0.1, 0, 0, 1.0])):
        fired, Wn = o.vacuum_guard(Sp_bad, vol, bad)
        rf = 1e-12 * 2.0
        assert fired and np.array_equal(Wn, np.array([rf, 0.0, 0.0, 0.5 * 3 * rf * 3.0]))
    fired, Wn = o.vacuum_guard(Sp, vol, np.array([np.nan, 0, 0, 1.0]))
    assert fired and np.array_equal(Wn, Sp / vol)


def test_vacuum_guard_fires_when_a_rarefaction_empties_a_cell():
    """Wave-only 1D: a thin low-density cell between two streams leaving it
    at twenty times the sound speed is emptied within one step; the step
    counts the guard and the cell holds the floor state exactly (no
    particles in wave-only runs), while its neighbours stay valid."""
    xs = np.linspace(0.0, 10.0, 11)
    m = wl.uniform1d(xs, rho=1.0, U=0.0, T=1.0, bc=wl.BC_SYMMETRY, mu_ref=1e-6)
    m["wave_only"] = 1
    W = m["W0"].copy()
    for i in range(10):
        U = -20.0 if i < 5 else 20.0
        rho = 1e-9 if i in (4, 5) else 1.0
        W[i] = wl.conservative(rho, U, 0.0, 1.0, 1)
    o = oracle.Oracle(m, W0=np.tile(wl.conservative(1.0, 0.0, 0.0, 1.0, 1), (10, 1)))
    o.set_fields(W)
    o.step(1)
    _, info = o.counts()
    Wn = o.fields()
    assert info["guard"] >= 1
    rf = 1e-12 * m["ref"]["rho_inf"]
    floor = np.array([rf, 0.0, 0.5 * 3 * rf * m["ref"]["T_inf"]])
    hit = [i for i in range(10) if np.array_equal(Wn[i], floor)]
    assert len(hit) == info["guard"] and set(hit) <= {3, 4, 5, 6}
    for i in range(10):
        rho, e = Wn[i, 0], Wn[i, 2] - 0.5 * Wn[i, 1] ** 2 / Wn[i, 0]
        assert rho > 0 and e > 0


# ---------------------------------------------------------------------------
# Shakhov sampler fallback
# ---------------------------------------------------------------------------

def _draw2(seed, pid, step, purpose, call):
    o = oracle.philox([pid & 0xFFFFFFFF, pid >> 32, step, (purpose << 24) | call], [seed & 0xFFFFFFFF, seed >> 32])
    return oracle.uniform(o[0], o[1]), oracle.uniform(o[2], o[3])


def _gauss3(seed, pid, step, call0):
    e0, e1 = _draw2(seed, pid, step, 2, call0)
    e2, e3 = _draw2(seed, pid, step, 2, call0 + 1)
    r0, r1 = math.sqrt(-2.0 * math.log(e0)), math.sqrt(-2.0 * math.log(e2))
    return [r0 * math.cos(2 * math.pi * e1), r0 * math.sin(2 * math.pi * e1), r1 * math.cos(2 * math.pi * e3)]


def test_shakhov_fallback_takes_the_first_draw_inside_the_cut():
    """With a heat flux so large that the acceptance bound B is ~10^3, most
    particles exhaust the 64 attempts.  Such a particle takes the deviation
    of its first attempt within c_max = 6 sqrt(R T^h) (recomputed here from
    the Philox stream): never a rejected draw outside the cut.  Accepted
    particles are unaffected by the reading."""
    m = wl.uniform1d(np.linspace(0, 1, 3), Pr=2.0 / 3.0)
    o = oracle.Oracle(m)
    seed = m["seed"]
    Uh, Th = [0.1, 0.0], 1.3
    shak = [0.0, 0.0, 1.0, 1.0, 400.0, 0.0]  # U, T, p of the cell, heat flux Q
    sig = math.sqrt(Th)
    n_capped = 0
    for j in range(200):
        pid = (7 << 44) | (1 << 20) | j
        z, capped = o.sample_deviation(pid, 7, Uh, Th, shak)
        if not capped:
            continue
        n_capped += 1
        first = None
        for att in range(64):
            zz = _gauss3(seed, pid, 7, 2 * att)
            if math.sqrt(zz[0] ** 2 + zz[1] ** 2 + zz[2] ** 2) * sig <= 6 * sig:
                first = zz
                break
        assert first is not None
        assert np.allclose(z, first, rtol=1e-14, atol=1e-15), (z, first)
        assert math.sqrt(z[0] ** 2 + z[1] ** 2 + z[2] ** 2) <= 6.0
    assert n_capped > 50
