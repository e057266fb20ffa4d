"""FP64 reference of the learned warm start (test infrastructure only).

Only the tests may import this module.  It restates, in plain numpy, what the
warm-start kernels of the product library compute:

  - the feature map: the steady field of a coarse wave-only solve on an
    O-grid, converted to normalized primitives p = (ln rho/rho_inf, u/U_inf,
    v/U_inf, ln T/T_inf), bilinearly interpolated in cell-index space onto a
    finer O-grid whose nodes include every coarse node (periodic in the
    angular index, clamped in the radial one), followed by the case
    parameters and a Fourier encoding of the cell-index coordinates;
  - a multilayer perceptron with GELU activations (GELU(z) = z Phi(z), Phi the
    standard normal distribution function), its backward pass for the mean
    squared error, and the Adam update (Kingma and Ba, 2015);
  - the decoding of the network output into a conservative initial field.

The paper (arXiv 2607.09552) defines none of this: its method starts from a
given initial field and fixes the local steps from it (Sec. IV, Eq. (33)).
Where the kernels round operands to BF16, the functions here take a `q`
argument that rounds at the same points (`bf16`), so the two can be compared
on identical quantized inputs; everything else is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_FEATURES = 32
N_OUT = 4
# case-parameter normalization: Ma in [5, 20], Kn in [0.005, 0.2] (log), T_w in [0.1, 0.5]
MA_C, MA_H = 12.5, 7.5
LKN_C, LKN_H = 0.5 * (math.log(0.005) + math.log(0.2)), 0.5 * math.log(40.0)
TW_C, TW_H = 0.3, 0.2


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.
    NaN stays NaN; the largest finite values round to infinity as IEEE does."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _ident(x):
    return x


def forward(params, X, q=_ident):
    """params: list of (W [out x in], b [out]); hidden layers GELU, the last
    linear.  Returns (Y, cache) with cache[l] = (layer input, Z)."""
    cache = []
    H = q(X)
    for l, (W, b) in enumerate(params):
        Z = H @ q(W).T + b
        cache.append((H, Z))
        H = gelu(Z) if l < len(params) - 1 else Z
        if l < len(params) - 1:
            H = q(H)
    return H, cache


def backward(params, cache, dY, q=_ident):
    """Gradients [(dW, db)] of a scalar loss whose gradient with respect to
    the network output is dY; also returns the gradient with respect to the
    input."""
    grads = [None] * len(params)
    G = dY
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        H, Z = cache[l]
        dZ = G * gelu_grad(Z) if l < len(params) - 1 else G
        dZq = q(dZ)
        grads[l] = (dZq.T @ H, dZ.sum(axis=0))
        G = dZq @ q(W)
    return grads, G


def mse(Y, T, n_out=N_OUT):
    """Loss sum((Y[:, :n_out] - T)^2) / (rows * n_out) and its gradient
    (zero on the padded output columns)."""
    M = Y.shape[0]
    d = Y[:, :n_out] - T
    g = np.zeros_like(Y)
    g[:, :n_out] = 2.0 * d / (M * n_out)
    return float((d * d).sum() / (M * n_out)), g


def adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step t >= 1; returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    w = w - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return w, m, v


def normalized_primitives(W, rho_inf, U_inf, T_inf, R=1.0, D=0):
    """Conservative 2D cell states [n x 4] -> (ln rho/rho_inf, u/U_inf,
    v/U_inf, ln T/T_inf) with rho E = rho |U|^2 / 2 + (3 + D) rho R T / 2."""
    rho = W[:, 0]
    u, v = W[:, 1] / rho, W[:, 2] / rho
    T = (W[:, 3] / rho - 0.5 * (u * u + v * v)) / (0.5 * (3 + D) * R)
    return np.stack([np.log(rho / rho_inf), u / U_inf, v / U_inf, np.log(T / T_inf)], axis=1)


def upsample(Pc, nct, ncr, nft, nfr):
    """Bilinear interpolation in cell-index space of coarse cell values Pc
    [ncr * nct x k] (cell (i, j) at row j * nct + i) onto the fine cells.
    Fine cell (I, J) sits at coarse index coordinates
    x = (I + 1/2) nct / nft - 1/2 (periodic) and y = (J + 1/2) ncr / nfr - 1/2
    (clamped to [0, ncr - 1])."""
    Pc = Pc.reshape(ncr, nct, -1)
    out = np.empty((nfr, nft, Pc.shape[2]))
    for J in range(nfr):
        y = min(max((J + 0.5) * ncr / nfr - 0.5, 0.0), ncr - 1.0)
        j0 = min(int(math.floor(y)), ncr - 2)
        b = y - j0
        for I in range(nft):
            x = (I + 0.5) * nct / nft - 0.5
            i0 = int(math.floor(x))
            a = x - i0
            i0m, i1m = i0 % nct, (i0 + 1) % nct
            out[J, I] = ((1 - a) * (1 - b) * Pc[j0, i0m] + a * (1 - b) * Pc[j0, i1m]
                         + (1 - a) * b * Pc[j0 + 1, i0m] + a * b * Pc[j0 + 1, i1m])
    return out.reshape(nfr * nft, -1)


def encoding(nft, nfr, Ma, Kn, Tw):
    """Columns 4..21 of the features of every fine cell: the normalized case
    parameters, sin/cos(2 pi k s) for k = 1..4 with s = (I + 1/2)/nft, 2 r - 1
    and sin/cos(pi k r) for k = 1..3 with r = (J + 1/2)/nfr."""
    I = np.tile(np.arange(nft), nfr)
    J = np.repeat(np.arange(nfr), nft)
    s = (I + 0.5) / nft
    r = (J + 0.5) / nfr
    cols = [np.full(I.shape, (Ma - MA_C) / MA_H), np.full(I.shape, (math.log(Kn) - LKN_C) / LKN_H),
            np.full(I.shape, (Tw - TW_C) / TW_H)]
    for k in range(1, 5):
        cols += [np.sin(2 * math.pi * k * s), np.cos(2 * math.pi * k * s)]
    cols.append(2.0 * r - 1.0)
    for k in range(1, 4):
        cols += [np.sin(math.pi * k * r), np.cos(math.pi * k * r)]
    return np.stack(cols, axis=1)


def features(Wc, nct, ncr, nft, nfr, case, rows=None):
    """Feature matrix [rows x 32] (FP64, before BF16 rounding) and the
    interpolated primitives P [n_fine x 4].  case = (Ma, Kn, T_w, rho_inf,
    U_inf, T_inf, R, D); rows beyond the fine cells are zero."""
    Ma, Kn, Tw, rho_inf, U_inf, T_inf, R, D = case
    nf = nft * nfr
    rows = nf if rows is None else rows
    P = upsample(normalized_primitives(Wc, rho_inf, U_inf, T_inf, R, D), nct, ncr, nft, nfr)
    X = np.zeros((rows, N_FEATURES))
    X[:nf, :4] = P
    X[:nf, 4:22] = encoding(nft, nfr, Ma, Kn, Tw)
    return X, P


def decode(Y, P, rho_inf, U_inf, T_inf, R=1.0, D=0):
    """Initial field from the network output: p = P + Y[:, :4]; conservative
    (rho, rho u, rho v, rho E)."""
    p = P + Y[: P.shape[0], :4]
    rho = rho_inf * np.exp(p[:, 0])
    u, v = U_inf * p[:, 1], U_inf * p[:, 2]
    T = T_inf * np.exp(p[:, 3])
    E = 0.5 * rho * (u * u + v * v) + 0.5 * (3 + D) * rho * R * T
    return np.stack([rho, rho * u, rho * v, E], axis=1)
