"""Whole-step pin of the oracle's reduction to the global-time-step scheme.

With every local time step equal (Eq. (34)), the LTS step of Sec. IV.B --
normalized per-side coefficients (Eqs. (47)-(48)), time-averaged fluxes
multiplied by each cell's dt in Eq. (53), particle mass and remaining time
scaled by dt_R/dt_L at crossings (Eqs. (41), (52)) -- must reduce to the GTS
UGKWP step of Sec. III: un-normalized coefficients of Eq. (16), time-integrated
fluxes, no scaling, Eq. (32) (the paper's last paragraph of Sec. IV.B).

The GTS step below is written independently in plain Python from Sec. III:
its own Philox4x32-10 (checked against the published known-answer vectors),
sampling, moment matching, 1D tracking with specular walls, exactly rounded
tallies (math.fsum), MUSCL/van Leer reconstruction, half-range moments from
erfc, the microslopes by solving the moment systems of Eqs. (20) and (22) as
4 x 4 linear systems, and the time-integrated fluxes of Eqs. (23) and (31).
A closed box with symmetry walls at both ends, Pr = 1, a non-uniform start.
The oracle run with lts = 0 must give identical particle ids, cells and
counts and the same fields and tallies to 1e-13 of each component's scale.
Planted in the oracle on the CPU and caught (field errors of 1e-2 and 1e-3
after one step): the two sides' relaxation times swapped in the face flux,
and the equilibrium slope off by a factor of two.
"""
import math
import os

import numpy as np

import oracle
import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M32 = 0xFFFFFFFF


# ---------------------------------------------------------------------------
# random numbers: Philox4x32-10 (Salmon et al., SC'11)
# ---------------------------------------------------------------------------

def philox(c, k):
    c0, c1, c2, c3 = c
    k0, k1 = k
    for _ in range(10):
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c3 ^ k1) & M32, p0 & M32
        k0 = (k0 + 0x9E3779B9) & M32
        k1 = (k1 + 0xBB67AE85) & M32
    return [c0, c1, c2, c3]


def test_python_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        assert philox(w[0:4], w[4:6]) == w[6:10]


def uniforms(seed, pid, step, purpose, call):
    o = philox([pid & M32, pid >> 32, step & M32, (purpose << 24) | call], [seed & M32, seed >> 32])
    u = lambda a, b: (((a << 20) | (b >> 12)) + 0.5) * 2.0 ** -52
    return u(o[0], o[1]), u(o[2], o[3])


FREE, POS, VEL = 0, 1, 2


def sq3(a):
    return (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]


def gauss3(seed, pid, step):
    e0, e1 = uniforms(seed, pid, step, VEL, 0)
    e2, e3 = uniforms(seed, pid, step, VEL, 1)
    r0, r1 = math.sqrt(-2.0 * math.log(e0)), math.sqrt(-2.0 * math.log(e2))
    a0, a1 = 2.0 * math.pi * e1, 2.0 * math.pi * e3
    return [r0 * math.cos(a0), r0 * math.sin(a0), r1 * math.cos(a1)]


# ---------------------------------------------------------------------------
# moments of a Maxwellian in the face frame (K lumped degrees of freedom)
# ---------------------------------------------------------------------------

def normal_moments(U, lam, half, kmax=8):
    """<u^k> over u > 0 (half = +1), u < 0 (-1) or all u (0), unit density."""
    M = [0.0] * (kmax + 1)
    if half == 0:
        M[0], M[1] = 1.0, U
    else:
        g = math.exp(-lam * U * U) / (2.0 * math.sqrt(math.pi * lam))
        M[0] = 0.5 * math.erfc(-half * math.sqrt(lam) * U)
        M[1] = U * M[0] + half * g
    for k in range(kmax - 1):
        M[k + 2] = U * M[k + 1] + (k + 1) / (2.0 * lam) * M[k]
    return M


def state(W, K):
    rho = W[0]
    U, V = W[1] / rho, W[2] / rho
    e = W[3] - 0.5 * rho * (U * U + V * V)
    return rho, U, V, (K + 2) * rho / (4.0 * e)


def moment_matrix(W, K, half, a):
    """E[q][r] = <u^a Psi_q phi_r> over the half (unit density), phi =
    (1, u, v, (u^2 + v^2 + xi^2)/2), for the Maxwellian of W (face frame)."""
    rho, U, V, lam = state(W, K)
    n = normal_moments(U, lam, half)
    t = [1.0, V]
    for k in range(3):
        t.append(V * t[k + 1] + (k + 1) / (2.0 * lam) * t[k])
    x = [1.0, K / (2.0 * lam), K * (K + 2) / (4.0 * lam * lam)]

    def m(p, q, d):
        return n[p] * t[q] * x[d]
    # a basis function as {(power u, power v, power xi^2): coefficient}
    basis = [{(0, 0, 0): 1.0}, {(1, 0, 0): 1.0}, {(0, 1, 0): 1.0},
             {(2, 0, 0): 0.5, (0, 2, 0): 0.5, (0, 0, 1): 0.5}]
    E = np.zeros((4, 4))
    for qi, pq in enumerate(basis):
        for ri, pr in enumerate(basis):
            s = 0.0
            for (p1, q1, d1), c1 in pq.items():
                for (p2, q2, d2), c2 in pr.items():
                    s += c1 * c2 * m(a + p1 + p2, q1 + q2, d1 + d2)
            E[qi, ri] = s
    return E


def psi_flux(W, K, half, c=None, a=1):
    """rho <u^a Psi (c . phi)> over the half; c None: phi = 1."""
    E = moment_matrix(W, K, half, a)
    cc = np.array([1.0, 0, 0, 0]) if c is None else np.asarray(c)
    return W[0] * (E @ cc)


def slope(W, dW, K):
    """Microslope coefficients c with rho <Psi g (c . phi)> = dW (Eq. (20))."""
    return np.linalg.solve(W[0] * moment_matrix(W, K, 0, 0), dW)


def delta(dt, tau):
    """Time integrals of Eq. (16), un-normalized."""
    E = math.exp(-dt / tau)
    return dict(a=dt - tau * (1 - E), b=2 * tau * tau * (1 - E) - tau * dt - tau * dt * E,
                c=0.5 * dt * dt - tau * dt + tau * tau * (1 - E), d=tau * (1 - E),
                e=tau * dt * E - tau * tau * (1 - E), E=E)


def valid(W):
    return W[0] > 0 and W[3] - 0.5 * W[0] * ((W[1] / W[0]) ** 2 + (W[2] / W[0]) ** 2) > 0


def recon(Wfar, xfar, Ws, xs, Wo, xo):
    """MUSCL along the normal with the van Leer limiter, distance-weighted
    one-sided differences; first order if no far cell or an invalid value."""
    if Wfar is None:
        return Ws.copy(), np.zeros(4)
    s = np.zeros(4)
    for q in range(4):
        d1 = (Ws[q] - Wfar[q]) / (xs - xfar)
        d2 = (Wo[q] - Ws[q]) / (xo - xs)
        p = d1 * d2
        s[q] = 2.0 * p / (d1 + d2) if p > 0 else 0.0
    v = Ws - s * xs
    return (v, s) if valid(v) else (Ws.copy(), np.zeros(4))


def gts_face_flux(WL, WR, dW0, HL, HR, sHL, sHR, dt, tauL, tauR, K):
    """Time-integrated flux over [0, dt], face frame: Eq. (23) integrated
    with per-side coefficients (Sec. III.A), plus Eq. (31) read upwind."""
    W0 = psi_flux(WL, K, +1, a=0) + psi_flux(WR, K, -1, a=0)
    F = np.zeros(4)
    if W0[0] > 0 and valid(W0):
        a = slope(W0, dW0, K)
        A = slope(W0, -psi_flux(W0, K, 0, a, a=1), K)
        for half, tau in ((+1, tauL), (-1, tauR)):
            d = delta(dt, tau)
            F += d["a"] * psi_flux(W0, K, half, a=1) + d["b"] * psi_flux(W0, K, half, a, a=2) \
                + d["c"] * psi_flux(W0, K, half, A, a=1)
    for half, tau, H, sH in ((+1, tauL, HL, sHL), (-1, tauR, HR, sHR)):
        if H is None:
            continue
        d = delta(dt, tau)
        ah = slope(H, sH, K)
        F += (d["d"] - dt * d["E"]) * psi_flux(H, K, half, a=1) \
            + (d["e"] + 0.5 * dt * dt * d["E"]) * psi_flux(H, K, half, ah, a=2)
    return F


# ---------------------------------------------------------------------------
# one GTS UGKWP step on a 1D closed box (symmetry faces at both ends)
# ---------------------------------------------------------------------------

class GtsBox:
    def __init__(self, m):
        self.x = m["nodes"][:, 0].copy()
        self.nc = len(self.x) - 1
        self.h = np.diff(self.x)
        self.c = 0.5 * (self.x[1:] + self.x[:-1])
        g = m["gas"]
        self.R, self.omega, self.mu, self.Tref = g["R"], g["omega"], g["mu_ref"], g["T_ref"]
        self.K = 1 + g["D"]
        self.nref, self.seed = m["n_ref"], m["seed"]
        self.W = m["W0"].copy()
        # Eq. (33) per cell, Eq. (34): the global step
        dts = []
        for i in range(self.nc):
            rho, U, T = self.prim(self.W[i])
            dts.append((m["cfl"] * self.h[i]) / ((abs(U) + 3.0 * math.sqrt(self.R * T)) * 2.0))
        self.dt = min(dts)
        self.P = []  # particles: [pid, cell, x, u0, u1, u2, m]
        self.n = 0

    def prim(self, W):
        rho = W[0]
        U = W[1] / rho
        e = W[2] - 0.5 * rho * U * U
        return rho, U, 2.0 * e / ((3 + self.K - 1) * self.R * rho)

    def tau(self, rho, T):
        return self.mu * (T / self.Tref) ** self.omega / (rho * self.R * T)

    @staticmethod
    def psi(p):
        u = p[3:6]
        return [p[6], p[6] * u[0], p[6] * (0.5 * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]))]

    def tally(self, parts):
        S = [[[] for _ in range(3)] for _ in range(self.nc)]
        for p in parts:
            for q, v in enumerate(self.psi(p)):
                S[p[1]][q].append(v)
        return np.array([[math.fsum(S[i][q]) for q in range(3)] for i in range(self.nc)])

    def frame(self, W, n):
        return np.array([W[0], W[1] * n, 0.0, W[2]])

    def step(self):
        nc, dt, n, K = self.nc, self.dt, self.n, self.K
        tau = np.array([self.tau(*self.prim(self.W[i])[::2]) for i in range(nc)])
        Sret = self.tally(self.P)
        Wh = self.W - Sret / self.h[:, None]
        hv = [Wh[i, 0] > 0 and Wh[i, 2] - 0.5 * Wh[i, 1] ** 2 / Wh[i, 0] > 0 for i in range(nc)]
        # free-transport times of the retained particles
        for p in self.P:
            e0, _ = uniforms(self.seed, p[0], n, FREE, 0)
            s = -tau[p[1]] * math.log(e0)
            p.append(s < dt)
            p.append(s if s < dt else dt)
        # new collisionless particles from the hydrodynamic wave, Eqs. (25)-(26)
        new = []
        for i in range(nc):
            if not hv[i]:
                continue
            E = math.exp(-(dt / tau[i]))
            rho_hp = Wh[i, 0] * E
            if not rho_hp > 0:
                continue
            N = math.ceil((rho_hp / self.W[i, 0]) * self.nref)
            mk = (rho_hp * self.h[i]) / N
            rh, Uh, Th = self.prim(Wh[i])
            sig = math.sqrt(self.R * Th)
            zs = []
            for j in range(N):
                pid = (n << 44) | (i << 20) | j
                e0, _ = uniforms(self.seed, pid, n, POS, 0)
                x = self.x[i] + e0 * (self.x[i + 1] - self.x[i])
                zs.append((pid, x, gauss3(self.seed, pid, n)))
            zm, alpha = [0.0, 0.0, 0.0], 1.0
            if N >= 2:
                zm = [math.fsum(z[2][d] for z in zs) / N for d in range(3)]
                S = math.fsum(sq3([z[2][d] - zm[d] for d in range(3)]) for z in zs)
                alpha = math.sqrt((3.0 * N) / S)
            for pid, x, z in zs:
                w = [(z[d] - zm[d]) * alpha for d in range(3)]
                new.append([pid, i, x, Uh + sig * w[0], sig * w[1], sig * w[2], mk, False, dt])
        pre = self.P + new
        Sm = self.tally(pre)
        # free transport, specular walls at both ends
        for p in pre:
            t = p[8]
            while True:
                i, x, u = p[1], p[2], p[3]
                if u > 0:
                    nrm, off = 1.0, self.x[i + 1]
                elif u < 0:
                    nrm, off = -1.0, -self.x[i]
                else:
                    p[2] = x + u * t
                    break
                te = (off - nrm * x) / (u * nrm)
                te = max(te, 0.0)
                if not te < t:
                    p[2] = x + u * t
                    break
                p[2] = x + u * te
                t = t - te
                j = i + (1 if u > 0 else -1)
                if 0 <= j < nc:
                    p[1] = j
                else:
                    p[3] = -u
        Sp = self.tally(pre)
        self.P = [p[:7] for p in pre if not p[7]]
        # wave fluxes, time-integrated; face k at node k, normal +x (cell
        # k-1 -> k); the end faces with a mirror ghost, normal out of the box
        dF = np.zeros((nc, 3))
        Wf = [self.frame(self.W[i], 1.0) for i in range(nc)]
        Hf = [self.frame(Wh[i], 1.0) for i in range(nc)]
        for k in range(1, nc):
            L, R = k - 1, k
            xf = self.x[k]
            xi = self.c - xf
            WLf, _ = recon(Wf[L - 1] if L >= 1 else None, xi[L - 1] if L >= 1 else 0.0, Wf[L], xi[L], Wf[R], xi[R])
            WRf, _ = recon(Wf[R + 1] if R + 1 < nc else None, xi[R + 1] if R + 1 < nc else 0.0, Wf[R], xi[R], Wf[L], xi[L])
            dW0 = (Wf[R] - Wf[L]) / (xi[R] - xi[L])
            HL = HR = None
            sHL = sHR = np.zeros(4)
            if hv[L]:
                far = L >= 1 and hv[L - 1] and hv[R]
                HL, sHL = recon(Hf[L - 1] if far else None, xi[L - 1] if far else 0.0, Hf[L], xi[L], Hf[R], xi[R])
            if hv[R]:
                far = R + 1 < nc and hv[R + 1] and hv[L]
                HR, sHR = recon(Hf[R + 1] if far else None, xi[R + 1] if far else 0.0, Hf[R], xi[R], Hf[L], xi[L])
            F = gts_face_flux(WLf, WRf, dW0, HL, HR, sHL, sHR, dt, tau[L], tau[R], K)
            Fx = np.array([F[0], F[1], F[3]])
            dF[L] += Fx
            dF[R] -= Fx
        for i, nrm, xf in ((0, -1.0, self.x[0]), (nc - 1, 1.0, self.x[nc])):
            wL, hL = self.frame(self.W[i], nrm), self.frame(Wh[i], nrm)
            wG, hG = wL * np.array([1, -1, 1, 1]), hL * np.array([1, -1, 1, 1])
            xL = (self.c[i] - xf) * nrm
            dW0 = (wG - wL) / (-2.0 * xL)
            F = gts_face_flux(wL, wG, dW0, hL if hv[i] else None, hG if hv[i] else None, np.zeros(4), np.zeros(4),
                              dt, tau[i], tau[i], K)
            dF[i] += np.array([F[0], F[1] * nrm, F[3]])
        # Eq. (32)
        self.W = self.W - dF / self.h[:, None] + (Sp - Sm) / self.h[:, None]
        self.n += 1
        return Sm, Sp


def test_lts_oracle_with_equal_steps_is_the_gts_step():
    x = np.concatenate([[0.0], np.cumsum(1.15 ** np.arange(7))])
    m = wl.uniform1d(x, rho=1.0, U=0.0, T=1.0, bc=wl.BC_SYMMETRY, mu_ref=0.5, n_ref=25, seed=7)
    nc = m["n_cells"]
    xc = 0.5 * (x[1:] + x[:-1])
    rho = 1.0 + 0.3 * np.sin(xc)
    U = 0.4 * np.cos(0.7 * xc)
    T = 1.0 + 0.2 * np.cos(xc)
    m["W0"] = np.stack([wl.conservative(r, u, 0.0, t, 1) for r, u, t in zip(rho, U, T)])
    m["lts"] = 0
    o = oracle.Oracle(m)
    g = GtsBox(m)
    assert np.allclose(o.dt(), g.dt, rtol=1e-15, atol=0)
    for n in range(1, 5):
        Sm, Sp = g.step()
        o.step(1)
        pr = o.particles()
        pid = np.array([p[0] for p in g.P], dtype=np.uint64)
        order = np.argsort(pid)
        assert np.array_equal(pid[order], pr["pid"]), n
        assert np.array_equal(np.array([p[1] for p in g.P])[order], pr["cell"]), n
        Wo = o.fields()
        scale = np.abs(Wo).max(axis=0)
        err = np.max(np.abs(g.W - Wo) / scale)
        assert err <= 1e-13, (n, err)
        Smo, Spo = o.tally()
        assert np.max(np.abs(Sm - Smo) / np.abs(Smo).max(axis=0)) <= 1e-13
        assert np.max(np.abs(Sp - Spo) / np.abs(Spo).max(axis=0)) <= 1e-13
        # advance both from the oracle's state so that rounding does not accumulate
        g.W = Wo.copy()
    assert len(g.P) > 50
