"""Seeded synthetic workloads: meshes, gas parameters and initial fields.

This module only builds inputs.  It holds none of the method's arithmetic and
is shared by the HIP product path, the CPU oracle, the tests and the bench.

A workload is a plain dict:

    dim         1 or 2
    nodes       float64 [n_nodes, dim]
    cell_ptr    int64 [n_cells + 1]     (2D only; CSR of CCW convex polygons)
    cell_nodes  int64 [cell_ptr[-1]]    (2D only)
    n_cells     int
    bface_nodes int64 [n_bfaces, dim]   node ids of each boundary face
    bface_type  int32 [n_bfaces]        BC_* below
    bface_data  float64 [n_bfaces, 8]   farfield: rho, ux, uy, T; wall: T_w
    gas         dict R, omega, mu_ref, T_ref, Pr, D
    cfl, n_ref, lts, seed
    ref         dict rho_inf, u_inf (2-vector), T_inf, L_ref  (surface coefficients)
    W0          float64 [n_cells, dim + 2]  conservative (rho, rho U, rho E)

Units are nondimensional with R = 1, rho_inf = 1, T_inf = 1 (freestream
reference state).  The mean free path follows the VHS model
(Bird): mu_inf = 15 rho sqrt(2 pi R T) lambda / (2 (5 - 2 w)(7 - 2 w)).
"""
from __future__ import annotations

import math

import numpy as np

BC_FARFIELD = 1
BC_OUTFLOW = 2
BC_WALL_DIFFUSE = 3
BC_SYMMETRY = 4
BC_WALL_MAXWELL = 6  # bface_data: T_w, accommodation alpha

GAMMA_MONATOMIC = 5.0 / 3.0


def vhs_mu(kn: float, l_ref: float, omega: float, rho: float = 1.0, T: float = 1.0, R: float = 1.0) -> float:
    """Viscosity giving VHS mean free path kn * l_ref at (rho, T)."""
    lam = kn * l_ref
    return 15.0 * rho * math.sqrt(2.0 * math.pi * R * T) * lam / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def conservative(rho, ux, uy, T, dim, D=0, R=1.0):
    """(rho, rho U, rho E) with rho E = rho |U|^2 / 2 + rho (3 + D) R T / 2."""
    rho = np.asarray(rho, dtype=np.float64)
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    if dim == 1:
        E = 0.5 * rho * ux * ux + 0.5 * (3 + D) * rho * R * T
        return np.stack(np.broadcast_arrays(rho, rho * ux, E), axis=-1)
    E = 0.5 * rho * (ux * ux + uy * uy) + 0.5 * (3 + D) * rho * R * T
    return np.stack(np.broadcast_arrays(rho, rho * ux, rho * uy, E), axis=-1)


def rankine_hugoniot(Ma: float, gamma: float = GAMMA_MONATOMIC):
    """Downstream (rho2, U2, T2) for upstream rho=1, T=1, U=Ma sqrt(gamma)."""
    U1 = Ma * math.sqrt(gamma)
    r = (gamma + 1) * Ma * Ma / ((gamma - 1) * Ma * Ma + 2)
    p = (2 * gamma * Ma * Ma - (gamma - 1)) / (gamma + 1)
    return r, U1 / r, p / r


def _bface_array(n):
    return np.zeros((n, 8), dtype=np.float64)


def _geometric_ratio(h1: float, n: int, length: float) -> float:
    """q with h1 (q^n - 1)/(q - 1) = length, by bisection."""
    if abs(h1 * n - length) < 1e-15 * length:
        return 1.0
    lo, hi = (1.0 + 1e-15, 2.0) if h1 * n < length else (1e-3, 1.0 - 1e-15)
    f = lambda q: h1 * (q ** n - 1.0) / (q - 1.0) - length
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (f(mid) > 0) == (f(hi) > 0):
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def base_params(**kw):
    p = dict(cfl=0.8, n_ref=200, lts=1, seed=1)
    p.update(kw)
    return p


# ----------------------------------------------------------------------------
# 1D meshes
# ----------------------------------------------------------------------------

def mesh1d(nodes_x, left_bc, right_bc, left_data=None, right_data=None):
    x = np.asarray(nodes_x, dtype=np.float64)
    bd = _bface_array(2)
    if left_data is not None:
        bd[0, : len(left_data)] = left_data
    if right_data is not None:
        bd[1, : len(right_data)] = right_data
    return dict(
        dim=1,
        nodes=x.reshape(-1, 1).copy(),
        n_cells=len(x) - 1,
        cell_ptr=None,
        cell_nodes=None,
        bface_nodes=np.array([[0], [len(x) - 1]], dtype=np.int64),
        bface_type=np.array([left_bc, right_bc], dtype=np.int32),
        bface_data=bd,
    )


def shock1d(n_half=50, ratio=1.03, h_min=1.0, Ma=3.0, Kn=0.05, omega=0.5, Pr=1.0,
            n_ref=200, lts=1, seed=1, cfl=0.8):
    """1D steady normal shock on a mesh graded by `ratio` toward x = 0.

    Cells k = 0..n_half-1 on each side have width h_min * ratio**k.  The
    freestream Knudsen number is defined on the smallest cell.  Both ends are
    far-field boundaries holding the Rankine-Hugoniot states; the initial
    field is the same step.
    """
    h = h_min * ratio ** np.arange(n_half)
    right = np.concatenate([[0.0], np.cumsum(h)])
    x = np.concatenate([-right[::-1], right[1:]])
    gamma = GAMMA_MONATOMIC
    U1 = Ma * math.sqrt(gamma)
    r2, U2, T2 = rankine_hugoniot(Ma, gamma)
    m = mesh1d(x, BC_FARFIELD, BC_FARFIELD, [1.0, U1, 0.0, 1.0], [r2, U2, 0.0, T2])
    xc = 0.5 * (x[1:] + x[:-1])
    up = xc < 0
    W0 = np.where(up[:, None], conservative(1.0, U1, 0.0, 1.0, 1), conservative(r2, U2, 0.0, T2, 1))
    m.update(
        name="shock1d",
        gas=dict(R=1.0, omega=omega, mu_ref=vhs_mu(Kn, h_min, omega), T_ref=1.0, Pr=Pr, D=0),
        ref=dict(rho_inf=1.0, u_inf=[U1, 0.0], T_inf=1.0, L_ref=h_min),
        W0=W0,
        **base_params(cfl=cfl, n_ref=n_ref, lts=lts, seed=seed),
    )
    return m


def uniform1d(x_nodes, rho=1.0, U=0.0, T=1.0, bc=BC_FARFIELD, mu_ref=1e-3, omega=0.5, Pr=1.0,
              n_ref=50, lts=1, seed=1, cfl=0.8, left=None, right=None):
    """A uniform state on an arbitrary 1D node list (test workloads)."""
    x = np.asarray(x_nodes, dtype=np.float64)
    left = left if left is not None else [rho, U, 0.0, T]
    right = right if right is not None else [rho, U, 0.0, T]
    m = mesh1d(x, bc if not isinstance(bc, tuple) else bc[0], bc if not isinstance(bc, tuple) else bc[1],
               left, right)
    n = len(x) - 1
    m.update(
        name="uniform1d",
        gas=dict(R=1.0, omega=omega, mu_ref=mu_ref, T_ref=1.0, Pr=Pr, D=0),
        ref=dict(rho_inf=rho, u_inf=[max(abs(U), 1.0), 0.0], T_inf=T, L_ref=1.0),
        W0=np.tile(conservative(rho, U, 0.0, T, 1), (n, 1)),
        **base_params(cfl=cfl, n_ref=n_ref, lts=lts, seed=seed),
    )
    return m


# ----------------------------------------------------------------------------
# 2D structured meshes stored as CCW quads
# ----------------------------------------------------------------------------

def _quads_from_grid(X, Y, ccw_check=True):
    """Cells of an (ni+1) x (nj+1) node grid; node id = j * (ni + 1) + i."""
    nj1, ni1 = X.shape
    ni, nj = ni1 - 1, nj1 - 1
    nodes = np.stack([X.ravel(), Y.ravel()], axis=1)
    I, J = np.meshgrid(np.arange(ni), np.arange(nj))
    n00 = J * ni1 + I
    quads = np.stack([n00, n00 + 1, n00 + 1 + ni1, n00 + ni1], axis=-1).reshape(-1, 4)
    return nodes, quads


def _orient_ccw(nodes, quads):
    p = nodes[quads]
    area = 0.5 * np.sum(p[:, :, 0] * np.roll(p[:, :, 1], -1, axis=1) - np.roll(p[:, :, 0], -1, axis=1) * p[:, :, 1], axis=1)
    flip = area < 0
    quads = quads.copy()
    quads[flip] = quads[flip][:, ::-1]
    return quads


def _finish2d(nodes, quads, bfaces, btype, bdata):
    quads = _orient_ccw(nodes, quads)
    n_cells = len(quads)
    return dict(
        dim=2,
        nodes=np.ascontiguousarray(nodes, dtype=np.float64),
        n_cells=n_cells,
        cell_ptr=np.arange(0, 4 * n_cells + 1, 4, dtype=np.int64),
        cell_nodes=np.ascontiguousarray(quads.ravel(), dtype=np.int64),
        bface_nodes=np.ascontiguousarray(bfaces, dtype=np.int64),
        bface_type=np.ascontiguousarray(btype, dtype=np.int32),
        bface_data=np.ascontiguousarray(bdata, dtype=np.float64),
    )


def box2d(xs, ys, bc=BC_SYMMETRY, bc_data=None):
    """Tensor-product box; every boundary face gets the same BC."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)
    nodes, quads = _quads_from_grid(X, Y)
    ni1 = len(xs)
    ni, nj = len(xs) - 1, len(ys) - 1
    bf = []
    for i in range(ni):
        bf.append((0 * ni1 + i, 0 * ni1 + i + 1))
        bf.append((nj * ni1 + i, nj * ni1 + i + 1))
    for j in range(nj):
        bf.append((j * ni1, (j + 1) * ni1))
        bf.append((j * ni1 + ni, (j + 1) * ni1 + ni))
    nb = len(bf)
    bd = _bface_array(nb)
    if bc_data is not None:
        bd[:, : len(bc_data)] = bc_data
    return _finish2d(nodes, quads, np.array(bf), np.full(nb, bc, dtype=np.int32), bd)


def ogrid(n_theta=200, n_r=150, r_in=1.0, r_out=15.0, h1=1e-4, theta0=math.pi):
    """O-grid around a unit cylinder: returns the mesh dict without physics.

    Node (i, j) sits at angle theta0 + 2 pi i / n_theta (so a node lies on the
    stagnation line) and radius r_j = r_in + h1 (q^j - 1)/(q - 1), with q
    solved so that r_{n_r} = r_out.  Cell (i, j) has id j * n_theta + i.
    Boundary faces: inner ring (wall) first, then the outer ring (far field).
    """
    q = _geometric_ratio(h1, n_r, r_out - r_in)
    j = np.arange(n_r + 1, dtype=np.float64)
    r = r_in + (h1 * j if q == 1.0 else h1 * (q ** j - 1.0) / (q - 1.0))
    r[-1] = r_out
    th = theta0 + 2.0 * math.pi * np.arange(n_theta) / n_theta
    R_, T_ = np.meshgrid(r, th, indexing="ij")  # [n_r+1, n_theta]
    nodes = np.stack([(R_ * np.cos(T_)).ravel(), (R_ * np.sin(T_)).ravel()], axis=1)
    nid = lambda i, jj: jj * n_theta + (i % n_theta)
    quads = []
    for jj in range(n_r):
        for i in range(n_theta):
            quads.append((nid(i, jj), nid(i, jj + 1), nid(i + 1, jj + 1), nid(i + 1, jj)))
    quads = np.array(quads, dtype=np.int64)
    bf = [(nid(i, 0), nid(i + 1, 0)) for i in range(n_theta)]
    bf += [(nid(i, n_r), nid(i + 1, n_r)) for i in range(n_theta)]
    return nodes, quads, np.array(bf, dtype=np.int64), q


def cylinder(n_theta=200, n_r=150, r_out=15.0, h1=1e-4, Ma=15.0, Kn=0.01, omega=0.81, Pr=2.0 / 3.0,
             Tw=0.2, n_ref=400, lts=1, seed=1, cfl=0.8):
    """Hypersonic flow past a cylinder of radius 1, diffuse isothermal wall."""
    nodes, quads, bf, q = ogrid(n_theta, n_r, 1.0, r_out, h1)
    U = Ma * math.sqrt(GAMMA_MONATOMIC)
    btype = np.array([BC_WALL_DIFFUSE] * n_theta + [BC_FARFIELD] * n_theta, dtype=np.int32)
    bd = _bface_array(len(bf))
    bd[:n_theta, 0] = Tw
    bd[n_theta:, :4] = [1.0, U, 0.0, 1.0]
    m = _finish2d(nodes, quads, bf, btype, bd)
    m.update(
        name="cylinder",
        stretch=q,
        n_theta=n_theta,
        n_r=n_r,
        gas=dict(R=1.0, omega=omega, mu_ref=vhs_mu(Kn, 1.0, omega), T_ref=1.0, Pr=Pr, D=0),
        ref=dict(rho_inf=1.0, u_inf=[U, 0.0], T_inf=1.0, L_ref=2.0),
        W0=np.tile(conservative(1.0, U, 0.0, 1.0, 2), (m["n_cells"], 1)),
        **base_params(cfl=cfl, n_ref=n_ref, lts=lts, seed=seed),
    )
    return m


def flat_plate(n_up=60, n_plate=240, n_y=200, up=0.25, height=0.5, h_x=1e-3, h_y=5e-5, Ma=10.0, Kn=0.0169,
               omega=0.74, Pr=1.0, Tw=1.0, n_ref=300, lts=1, seed=1, cfl=0.8):
    """Hypersonic flow over a flat plate of length 1 with a sharp leading edge
    at x = 0: x in [-up, 1], y in [0, height]; cells graded geometrically away
    from the leading edge (first width h_x on both sides) and from the wall
    (first height h_y).  Inflow (fixed freestream) on the left, far field on
    top, zero-gradient outflow on the right, symmetry on y = 0 for x < 0 and an
    isothermal diffuse wall on the plate."""
    qu = _geometric_ratio(h_x, n_up, up)
    qp = _geometric_ratio(h_x, n_plate, 1.0)
    qy = _geometric_ratio(h_y, n_y, height)
    xu = -graded(n_up, qu, h_x)[::-1]
    xp = graded(n_plate, qp, h_x)
    xs = np.concatenate([xu, xp[1:]])
    ys = graded(n_y, qy, h_y)
    X, Y = np.meshgrid(xs, ys)
    nodes, quads = _quads_from_grid(X, Y)
    ni1 = len(xs)
    ni, nj = len(xs) - 1, len(ys) - 1
    U = Ma * math.sqrt(GAMMA_MONATOMIC)
    bf, bt, bd = [], [], []
    free = [1.0, U, 0.0, 1.0]
    for i in range(ni):  # bottom: symmetry upstream, wall on the plate
        bf.append((i, i + 1))
        if i < n_up:
            bt.append(BC_SYMMETRY)
            bd.append([0.0] * 4)
        else:
            bt.append(BC_WALL_DIFFUSE)
            bd.append([Tw, 0.0, 0.0, 0.0])
    for i in range(ni):  # top: far field
        bf.append((nj * ni1 + i, nj * ni1 + i + 1))
        bt.append(BC_FARFIELD)
        bd.append(free)
    for j in range(nj):  # left: inflow; right: outflow
        bf.append((j * ni1, (j + 1) * ni1))
        bt.append(BC_FARFIELD)
        bd.append(free)
        bf.append((j * ni1 + ni, (j + 1) * ni1 + ni))
        bt.append(BC_OUTFLOW)
        bd.append([0.0] * 4)
    data = _bface_array(len(bf))
    data[:, :4] = np.array(bd)
    m = _finish2d(nodes, quads, np.array(bf), np.array(bt, dtype=np.int32), data)
    m.update(
        name="flat_plate",
        stretch=(qu, qp, qy),
        gas=dict(R=1.0, omega=omega, mu_ref=vhs_mu(Kn, 1.0, omega), T_ref=1.0, Pr=Pr, D=0),
        ref=dict(rho_inf=1.0, u_inf=[U, 0.0], T_inf=1.0, L_ref=1.0),
        W0=np.tile(conservative(1.0, U, 0.0, 1.0, 2), (m["n_cells"], 1)),
        **base_params(cfl=cfl, n_ref=n_ref, lts=lts, seed=seed),
    )
    return m


def cylinder_batch(n_cases=64, seed=2, n_ref=200, omega=0.81, Pr=2.0 / 3.0, lts=1, size=1.0):
    """Independent cylinder cases of uneven size and flow: case k draws
    u0..u3 uniform in [0, 1) (numpy generator seeded with `seed`):
    s = 1 + 2 u0 gives an (80 s) x (60 s) O-grid (scaled by `size`),
    Ma = 5 + 15 u1, Kn = 0.005 * 40^u2, T_w = 0.1 + 0.4 u3; Philox seed
    1000 + k.  Otherwise as `cylinder`."""
    rng = np.random.default_rng(seed)
    u = rng.random((n_cases, 4))
    cases = []
    for k in range(n_cases):
        s_ = 1.0 + 2.0 * u[k, 0]
        nt = max(8, int(round(80 * s_ * size)))
        nr = max(6, int(round(60 * s_ * size)))
        m = cylinder(n_theta=nt, n_r=nr, Ma=5.0 + 15.0 * u[k, 1], Kn=0.005 * 40.0 ** u[k, 2], omega=omega, Pr=Pr,
                     Tw=0.1 + 0.4 * u[k, 3], n_ref=n_ref, lts=lts, seed=1000 + k)
        cases.append(m)
    return cases


def with_maxwell_walls(m, alpha):
    """A copy of workload m whose diffuse walls become Maxwell walls with
    accommodation alpha (same wall temperature)."""
    w = dict(m)
    bt = m["bface_type"].copy()
    bd = m["bface_data"].copy()
    sel = bt == BC_WALL_DIFFUSE
    bt[sel] = BC_WALL_MAXWELL
    bd[sel, 1] = alpha
    w["bface_type"], w["bface_data"] = bt, bd
    return w


def with_internal_dof(m, D):
    """A copy of workload m for a gas with D internal degrees of freedom: the
    same density, velocity and temperature fields (the energy gains
    D rho R T / 2)."""
    w = dict(m)
    w["gas"] = dict(m["gas"], D=D)
    W = np.asarray(m["W0"], dtype=np.float64)
    dim = int(m["dim"])
    R = m["gas"]["R"]
    D0 = m["gas"]["D"]
    rho = W[:, 0]
    u = W[:, 1] / rho
    v = W[:, 2] / rho if dim == 2 else np.zeros_like(rho)
    ke = 0.5 * (u * u + v * v)
    T = (W[:, -1] / rho - ke) / (0.5 * (3 + D0) * R)
    w["W0"] = conservative(rho, u, v, T, dim, D=D, R=R)
    return w


def uniform2d(mesh, rho=1.0, ux=0.0, uy=0.0, T=1.0, mu_ref=1e-3, omega=0.5, Pr=1.0, n_ref=50,
              lts=1, seed=1, cfl=0.8):
    m = dict(mesh)
    m.update(
        name="uniform2d",
        gas=dict(R=1.0, omega=omega, mu_ref=mu_ref, T_ref=1.0, Pr=Pr, D=0),
        ref=dict(rho_inf=rho, u_inf=[max(math.hypot(ux, uy), 1.0), 0.0], T_inf=T, L_ref=1.0),
        W0=np.tile(conservative(rho, ux, uy, T, 2), (mesh["n_cells"], 1)),
        **base_params(cfl=cfl, n_ref=n_ref, lts=lts, seed=seed),
    )
    return m


def _polygon_mesh(nodes, polys, bc, bc_data=None):
    """Mesh of CCW convex polygons (lists of node ids); every open edge is a
    boundary face of type bc."""
    edges = {}
    for k, poly in enumerate(polys):
        for a, b in zip(poly, poly[1:] + poly[:1]):
            key = (min(a, b), max(a, b))
            edges[key] = edges.get(key, 0) + 1
    bf = [e for e, n in edges.items() if n == 1]
    bd = _bface_array(len(bf))
    if bc_data is not None:
        bd[:, : len(bc_data)] = bc_data
    ptr = np.zeros(len(polys) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(p) for p in polys])
    return dict(
        dim=2,
        nodes=np.ascontiguousarray(nodes, dtype=np.float64),
        n_cells=len(polys),
        cell_ptr=ptr,
        cell_nodes=np.array([i for p in polys for i in p], dtype=np.int64),
        bface_nodes=np.array(bf, dtype=np.int64).reshape(-1, 2),
        bface_type=np.full(len(bf), bc, dtype=np.int32),
        bface_data=bd,
    )


def triangulated_box(xs, ys, bc=BC_FARFIELD, bc_data=None, mixed=False):
    """Tensor-product box with every quad split into two triangles along
    alternating diagonals; with mixed=True only every other quad is split
    (triangles and quadrilaterals in one mesh)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)
    nodes = np.stack([X.ravel(), Y.ravel()], axis=1)
    ni1 = len(xs)
    polys = []
    for j in range(len(ys) - 1):
        for i in range(len(xs) - 1):
            a, b = j * ni1 + i, j * ni1 + i + 1
            c, d = b + ni1, a + ni1
            if mixed and (i + j) % 2 == 0:
                polys.append([a, b, c, d])
            elif (i + j) % 2 == 0:
                polys += [[a, b, c], [a, c, d]]
            else:
                polys += [[a, b, d], [b, c, d]]
    return _polygon_mesh(nodes, polys, bc, bc_data)


def honeycomb_box(nx, ny, h=1.0, bc=BC_FARFIELD, bc_data=None):
    """Regular hexagons of side h clipped to the box [0, W] x [0, H] spanned
    by nx x ny of them: hexagons inside, clipped convex polygons of 3 to 6
    vertices at the edges."""
    w = math.sqrt(3.0) * h
    W, H = nx * w, ny * 1.5 * h
    pts, polys = {}, []

    def node(x, y):
        key = (round(x, 9), round(y, 9))
        if key not in pts:
            pts[key] = len(pts)
        return pts[key]

    def clip(poly):
        for axis, lim, keep_le in ((0, 0.0, False), (0, W, True), (1, 0.0, False), (1, H, True)):
            out = []
            for k in range(len(poly)):
                p, q = poly[k], poly[(k + 1) % len(poly)]
                pin = p[axis] <= lim + 1e-12 if keep_le else p[axis] >= lim - 1e-12
                qin = q[axis] <= lim + 1e-12 if keep_le else q[axis] >= lim - 1e-12
                if pin:
                    out.append(p)
                if pin != qin:
                    t = (lim - p[axis]) / (q[axis] - p[axis])
                    r = [p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])]
                    r[axis] = lim
                    out.append(tuple(r))
            poly = out
            if not poly:
                return []
        # drop repeated and collinear vertices
        res = []
        for k in range(len(poly)):
            p0, p1, p2 = poly[k - 1], poly[k], poly[(k + 1) % len(poly)]
            cross = (p1[0] - p0[0]) * (p2[1] - p1[1]) - (p1[1] - p0[1]) * (p2[0] - p1[0])
            if abs(cross) > 1e-12 * h * h:
                res.append(p1)
        return res

    for r in range(-1, ny + 2):
        for c in range(-1, nx + 2):
            cx = c * w + (w / 2 if r % 2 else 0.0)
            cy = r * 1.5 * h
            hexa = [(cx + h * math.cos(math.pi / 6 + k * math.pi / 3), cy + h * math.sin(math.pi / 6 + k * math.pi / 3))
                    for k in range(6)]
            poly = clip(hexa)
            if len(poly) >= 3:
                area = 0.5 * sum(poly[k][0] * poly[(k + 1) % len(poly)][1] - poly[(k + 1) % len(poly)][0] * poly[k][1]
                                 for k in range(len(poly)))
                if area > 1e-6 * h * h:
                    polys.append([node(x, y) for x, y in poly])
    nodes = np.zeros((len(pts), 2))
    for (x, y), k in pts.items():
        nodes[k] = (x, y)
    return _polygon_mesh(nodes, polys, bc, bc_data)


def graded(n, ratio, h0=1.0):
    """Node coordinates 0, h0, h0 + h0 r, ... (n cells, geometric widths)."""
    h = h0 * ratio ** np.arange(n)
    return np.concatenate([[0.0], np.cumsum(h)])


def perturbed_field(m, amp=0.05, seed=0):
    """A smooth, seeded perturbation of a workload's W0 (test inputs)."""
    rng = np.random.default_rng(seed)
    W = m["W0"].copy()
    n = W.shape[0]
    f = 1.0 + amp * np.sin(np.linspace(0.0, 6.0, n) + rng.uniform(0, 6.28))
    W *= f[:, None]
    return W
