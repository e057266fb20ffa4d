"""Whole-step pins of the oracle in two more limits where the answer is known.

- collisionless limit (tau -> infinity) on a body: a flat plate at zero
  incidence with a diffuse isothermal wall in a free-molecular stream; the
  wall pressure, shear and heat flux are those of the incident freestream
  half-range Maxwellian plus the re-emitted wall Maxwellian (closed forms);
- equilibrium with particles: a uniform Maxwellian at rest in a closed
  specular box, advanced with both waves and particles, stays there in
  expectation (E[W^n - W^0] = 0 over seeds, for every cell and component).
"""
import math

import numpy as np

import oracle
import workloads as wl


def _plate_box(nx_up=5, nx_plate=10, nx_down=5, ny=10, h=0.1, Ma=2.0, Tw=1.5, n_ref=300, seed=5):
    """Uniform mesh x in [-nx_up h, (nx_plate + nx_down) h], y in [0, ny h];
    the plate x in [0, nx_plate h] on y = 0 is a diffuse wall at T_w, the rest
    of y = 0 a symmetry plane, every other side the free stream (rho = T = 1,
    U = Ma sqrt(5/3) along x); mu_ref so large that tau ~ 10^5 dt."""
    xs = h * np.arange(-nx_up, nx_plate + nx_down + 1, dtype=np.float64)
    ys = h * np.arange(0, ny + 1, dtype=np.float64)
    U = Ma * math.sqrt(5.0 / 3.0)
    box = wl.box2d(xs, ys, wl.BC_FARFIELD, [1.0, U, 0.0, 1.0])
    ni = len(xs) - 1
    bt = box["bface_type"].copy()
    bd = box["bface_data"].copy()
    walls = []
    for i in range(ni):  # bottom faces come first in pairs (bottom, top) per column
        b = 2 * i
        xc = 0.5 * (xs[i] + xs[i + 1])
        if 0.0 < xc < nx_plate * h:
            bt[b] = wl.BC_WALL_DIFFUSE
            bd[b, :4] = [Tw, 0.0, 0.0, 0.0]
            walls.append(b)
        else:
            bt[b] = wl.BC_SYMMETRY
            bd[b, :4] = 0.0
    box["bface_type"], box["bface_data"] = bt, bd
    m = wl.uniform2d(box, rho=1.0, ux=U, uy=0.0, T=1.0, mu_ref=1e3, n_ref=n_ref, seed=seed)
    m["ref"] = dict(rho_inf=1.0, u_inf=[U, 0.0], T_inf=1.0, L_ref=1.0)
    return m, U, Tw


def test_collisionless_flat_plate_free_molecular_wall_fluxes():
    """tau -> infinity, diffuse plate at T_w = 1.5 in a Ma 2 stream: the gas
    reaching the plate's top is the undisturbed free stream (re-emitted
    particles leave upward and never return, the symmetry plane mirrors a
    stream with no normal velocity onto itself), so per unit area
      p   = rho R T / 2 (1 + sqrt(T_w / T)),
      tau = rho U sqrt(R T / (2 pi)),
      q   = rho sqrt(R T / (2 pi)) (U^2 / 2 + 2 R (T - T_w)),
    the incident half-range Maxwellian plus the flux-weighted wall
    Maxwellian that re-emits the same mass.  Time and plate averages within
    five standard errors (batch means).  A re-emission at the gas
    temperature, a lost re-emitted momentum or a wrong slab flux of the far
    field moves one of them by 10 standard errors or more."""
    m, U, Tw = _plate_box()
    o = oracle.Oracle(m)
    o.step(150)
    rows = []
    for _ in range(450):
        o.step(1)
        s, _ = o.surface(0)
        rows.append(s[:, 3:6].copy())
    a = np.array(rows)  # steps x wall faces x (C_p, C_F, C_Q)
    qd = 0.5 * U * U
    p = a[:, :, 0] * qd + 1.0
    tau = a[:, :, 1] * qd
    q = a[:, :, 2] * qd * U
    series = np.stack([p.mean(1), tau.mean(1), q.mean(1)], axis=1)
    nb = 15
    bm = series.reshape(nb, -1, 3).mean(1)
    mean = series.mean(0)
    se = bm.std(0, ddof=1) / math.sqrt(nb)
    gam = math.sqrt(1.0 / (2.0 * math.pi))
    ref = np.array([0.5 * (1.0 + math.sqrt(Tw)), U * gam, gam * (0.5 * U * U + 2.0 * (1.0 - Tw))])
    z = (mean - ref) / se
    assert np.all(np.abs(z) < 5.0), (mean, ref, se, z)
    assert np.all(se < 0.02 * np.abs(ref)), se


def test_equilibrium_with_particles_is_preserved_in_expectation():
    """A uniform Maxwellian at rest in a closed specular box on a graded LTS
    mesh with dt/tau between 0.3 and 3 (waves and particles both carry gas):
    over 120 seeds, the change W^40 - W^0 of every cell and component has
    mean zero within five standard errors.  Planted on the CPU and caught:
    crossings that do not scale the particle mass by dt_R/dt_L (Eq. (41)),
    and a W^{p,+} tally that leaves out the collided particles (Eq. (30)).
    (A flux error common to both sides of every face cancels in a uniform
    state; the flux pins cover those.)"""
    x = wl.graded(8, 1.3)
    runs = []
    for seed in range(120):
        m = wl.uniform1d(x, rho=1.0, U=0.0, T=1.0, bc=wl.BC_SYMMETRY, mu_ref=0.3, n_ref=60, seed=100 + seed)
        o = oracle.Oracle(m)
        W0 = o.fields()
        o.step(40)
        runs.append(o.fields() - W0)
        o.close()
    d = np.array(runs)  # seeds x cells x components
    mean = d.mean(0)
    se = d.std(0, ddof=1) / math.sqrt(d.shape[0])
    z = mean / np.maximum(se, 1e-300)
    assert np.all(np.abs(z) < 5.0), z
    # the runs do fluctuate: the test has power
    assert np.all(se[:, 0] > 0)
