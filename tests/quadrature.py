"""Brute-force velocity-space quadrature used to pin the oracle's closed forms.

Independent of the oracle: it integrates the Maxwellian of Eq. (1) numerically
(Gauss-Legendre along u_n, split at u_n = 0; Gauss-Hermite along u_t;
generalized Gauss-Laguerre for the K lumped degrees of freedom), and solves the
moment systems of Eqs. (20) and (22) as plain 4x4 linear systems.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_genlaguerre, roots_hermite, roots_legendre

_NL, _NH, _NX = 160, 24, 24


def grid(U, V, lam, K, half):
    """Nodes/weights of the probability measure of a unit-density Maxwellian
    restricted to u_n > 0 (half=+1), u_n < 0 (-1) or all u_n (0).
    Returns un, ut, xi2, w (broadcast 3D arrays)."""
    sig = math.sqrt(0.5 / lam)
    lo, hi = U - 16 * sig, U + 16 * sig
    if half > 0:
        lo = max(lo, 0.0)
    elif half < 0:
        hi = min(hi, 0.0)
    if hi <= lo:
        z = np.zeros((1, 1, 1))
        return z, z, z, z
    xl, wl = roots_legendre(_NL)
    # split the interval at the mean for accuracy when it is inside
    pieces = [(lo, hi)] if not (lo < U < hi) else [(lo, U), (U, hi)]
    un_list, wn_list = [], []
    for a, b in pieces:
        un_list.append(0.5 * (b - a) * xl + 0.5 * (a + b))
        wn_list.append(0.5 * (b - a) * wl)
    un = np.concatenate(un_list)
    wn = np.concatenate(wn_list) * math.sqrt(lam / math.pi) * np.exp(-lam * (un - U) ** 2)
    xh, wh = roots_hermite(_NH)
    ut = V + xh / math.sqrt(lam)
    wt = wh / math.sqrt(math.pi)
    alpha = 0.5 * K - 1.0
    xs, ws = roots_genlaguerre(_NX, alpha)
    xi2 = xs / lam
    wx = ws / math.gamma(alpha + 1.0)
    UN, UT, XI = np.meshgrid(un, ut, xi2, indexing="ij")
    Wt = wn[:, None, None] * wt[None, :, None] * wx[None, None, :]
    return UN, UT, XI, Wt


def psi(un, ut, xi2):
    return np.stack([np.ones_like(un), un, ut, 0.5 * (un * un + ut * ut + xi2)])


def state(W, K):
    rho = W[0]
    U, V = W[1] / rho, W[2] / rho
    e = W[3] - 0.5 * rho * (U * U + V * V)
    lam = (K + 2) * rho / (4 * e)
    return rho, U, V, lam


def moment(W, K, half, fn=None, power=0):
    """rho * <u_n^power Psi fn(u)> over the chosen half for the Maxwellian of W."""
    rho, U, V, lam = state(W, K)
    un, ut, xi2, w = grid(U, V, lam, K, half)
    f = np.ones_like(un) if fn is None else fn(un, ut, xi2)
    return rho * np.sum(psi(un, ut, xi2) * (un ** power) * f * w, axis=(1, 2, 3))


def basis(un, ut, xi2):
    return [np.ones_like(un), un, ut, 0.5 * (un * un + ut * ut + xi2)]


def solve_slope(W, rhs, K):
    """Coefficients c of c0 + cn u_n + ct u_t + c4 (u^2 + xi^2)/2 with
    <Psi g (that polynomial)> = rhs (the moment systems of Eqs. (20), (22))."""
    rho, U, V, lam = state(W, K)
    un, ut, xi2, w = grid(U, V, lam, K, 0)
    P = psi(un, ut, xi2)
    B = basis(un, ut, xi2)
    M = np.array([[rho * np.sum(P[q] * B[r] * w) for r in range(4)] for q in range(4)])
    return np.linalg.solve(M, rhs)


def poly(c):
    return lambda un, ut, xi2: c[0] + c[1] * un + c[2] * ut + c[3] * 0.5 * (un * un + ut * ut + xi2)


def maxwell_W(rho, U, V, T, K, R=1.0):
    """Conservative face-frame W of a Maxwellian: rho E = rho(U^2+V^2)/2 + (K+2) rho R T / 2."""
    return np.array([rho, rho * U, rho * V, 0.5 * rho * (U * U + V * V) + 0.5 * (K + 2) * rho * R * T])


def delta_coeffs(dt, tau):
    """Eq. (16) written out (un-normalized)."""
    E = math.exp(-dt / tau)
    da = dt - tau * (1 - E)
    db = 2 * tau * tau * (1 - E) - tau * dt - tau * dt * E
    dc = 0.5 * dt * dt - tau * dt + tau * tau * (1 - E)
    dd = tau * (1 - E)
    de = tau * dt * E - tau * tau * (1 - E)
    return da, db, dc, dd, de, E
