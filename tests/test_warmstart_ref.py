"""Pins of the FP64 warm-start reference (oracle/warmstart_ref.py) against
closed forms, textbook values, finite differences and library routines."""
import math

import numpy as np
import torch

from oracle import warmstart_ref as ref
import workloads


def test_bf16_rounding_ties_to_even_and_matches_torch():
    # exact values, ties to even, just above a tie
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 0.0, 65504.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 0.0, 65536.0])
    assert np.array_equal(ref.bf16(x), want)
    r = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    t = torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ref.bf16(r), t)


def test_gelu_closed_forms():
    # GELU(z) = z Phi(z): Phi(1) = 0.8413447460685429 (normal table)
    assert ref.gelu(np.array(0.0)) == 0.0
    assert abs(ref.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(ref.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    z = np.linspace(-6, 6, 101)
    assert np.allclose(ref.gelu(z) - ref.gelu(-z), z, atol=1e-14, rtol=0)  # Phi(z) + Phi(-z) = 1
    tz = torch.nn.functional.gelu(torch.tensor(z)).numpy()
    assert np.allclose(ref.gelu(z), tz, atol=1e-15, rtol=0)


def test_gelu_grad_finite_differences():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (ref.gelu(z + h) - ref.gelu(z - h)) / (2 * h)
    assert np.allclose(ref.gelu_grad(z), fd, atol=1e-9, rtol=0)
    assert ref.gelu_grad(np.array(0.0)) == 0.5


def _tiny(seed=0, widths=(5, 7, 6, 3)):
    g = np.random.default_rng(seed)
    params = [(g.standard_normal((o, i)), g.standard_normal(o)) for i, o in zip(widths[:-1], widths[1:])]
    X = g.standard_normal((9, widths[0]))
    T = g.standard_normal((9, 2))
    return params, X, T


def _loss(params, X, T):
    Y, _ = ref.forward(params, X)
    return ref.mse(Y, T, n_out=2)[0]


def test_backward_matches_central_differences():
    params, X, T = _tiny()
    Y, cache = ref.forward(params, X)
    _, dY = ref.mse(Y, T, n_out=2)
    grads, dX = ref.backward(params, cache, dY)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = _loss(params, X, T)
                arr[idx] = old - h
                lm = _loss(params, X, T)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.allclose(g, fd, atol=1e-8, rtol=1e-6), l
    fd = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        old = X[idx]
        X[idx] = old + h
        lp = _loss(params, X, T)
        X[idx] = old - h
        lm = _loss(params, X, T)
        X[idx] = old
        fd[idx] = (lp - lm) / (2 * h)
    assert np.allclose(dX, fd, atol=1e-8, rtol=1e-6)


def test_backward_matches_torch_autograd():
    params, X, T = _tiny(seed=3, widths=(6, 16, 16, 4))
    Y, cache = ref.forward(params, X)
    _, dY = ref.mse(Y, T, n_out=2)
    grads, _ = ref.backward(params, cache, dY)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    h = torch.tensor(X)
    for l, (W, b) in enumerate(tp):
        h = h @ W.T + b
        if l < len(tp) - 1:
            h = torch.nn.functional.gelu(h)
    loss = ((h[:, :2] - torch.tensor(T)) ** 2).mean()
    loss.backward()
    for (gW, gb), (W, b) in zip(grads, tp):
        assert np.allclose(gW, W.grad.numpy(), atol=1e-12, rtol=1e-10)
        assert np.allclose(gb, b.grad.numpy(), atol=1e-12, rtol=1e-10)


def test_adam_first_step_and_torch():
    g = np.random.default_rng(2)
    w0, grad = g.standard_normal(50), g.standard_normal(50)
    # step 1: bias-corrected m = g, v = g^2, so the move is lr g / (|g| + eps)
    w1, m, v = ref.adam(w0, np.zeros(50), np.zeros(50), grad, 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w0 - 0.01 * np.sign(grad), atol=1e-15, rtol=0)
    # several steps against torch.optim.Adam
    tw = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([tw], lr=0.003, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        gt = g.standard_normal(50)
        opt.zero_grad()
        tw.grad = torch.tensor(gt)
        opt.step()
        w, m, v = ref.adam(w, m, v, gt, t, lr=0.003)
    assert np.allclose(w, tw.detach().numpy(), atol=1e-14, rtol=1e-12)


def test_upsample_reproduces_index_linear_fields():
    nct, ncr, nft, nfr = 8, 6, 40, 30
    i = np.tile(np.arange(nct), ncr).astype(float)
    j = np.repeat(np.arange(ncr), nct).astype(float)
    # constant
    assert np.allclose(ref.upsample(np.full((nct * ncr, 1), 2.5), nct, ncr, nft, nfr), 2.5, atol=1e-15)
    # linear in the radial index: exact, clamped at the first and last centres
    up = ref.upsample((3.0 + 0.5 * j)[:, None], nct, ncr, nft, nfr)[:, 0]
    J = np.repeat(np.arange(nfr), nft)
    y = np.clip((J + 0.5) * ncr / nfr - 0.5, 0, ncr - 1)
    assert np.allclose(up, 3.0 + 0.5 * y, atol=1e-14, rtol=0)
    # linear in the angular index, with the periodic wrap between the last
    # and first coarse columns
    up = ref.upsample(i[:, None], nct, ncr, nft, nfr)[:, 0].reshape(nfr, nft)
    # fine column 0 lies at coarse x = 0.5*8/40 - 0.5 = -0.4: 0.4 of column 7, 0.6 of column 0
    assert abs(up[0, 0] - 0.4 * 7) < 1e-14
    I = np.arange(nft)
    x = (I + 0.5) * nct / nft - 0.5
    inner = (x >= 0) & (x <= nct - 1)
    assert np.allclose(up[3, inner], x[inner], atol=1e-13)
    # coincident centres: fine cell (5 i + 2, 5 j + 2) is coarse cell (i, j)
    vals = np.random.default_rng(0).standard_normal((nct * ncr, 4))
    up = ref.upsample(vals, nct, ncr, nft, nfr).reshape(nfr, nft, 4)
    for (ic, jc) in ((0, 0), (3, 2), (7, 5)):
        assert np.allclose(up[5 * jc + 2, 5 * ic + 2], vals[jc * nct + ic], atol=1e-14, rtol=0)


def test_primitives_decode_round_trip():
    g = np.random.default_rng(4)
    n = 100
    rho, ux, uy, T = g.uniform(0.1, 5, n), g.normal(0, 3, n), g.normal(0, 3, n), g.uniform(0.2, 40, n)
    W = workloads.conservative(rho, ux, uy, T, 2)
    P = ref.normalized_primitives(W, 1.0, 6.0, 1.0)
    assert np.allclose(P, np.stack([np.log(rho), ux / 6, uy / 6, np.log(T)], axis=1), atol=1e-13)
    W2 = ref.decode(np.zeros((n, 32)), P, 1.0, 6.0, 1.0)
    assert np.allclose(W2, W, rtol=1e-13, atol=1e-13)


def test_encoding_columns():
    E = ref.encoding(40, 30, 12.5, math.sqrt(0.005 * 0.2), 0.3)
    assert E.shape == (1200, 18)
    assert np.allclose(E[:, :3], 0.0, atol=1e-15)  # the centre of every parameter range
    for k in range(4):
        s, c = E[:, 3 + 2 * k], E[:, 4 + 2 * k]
        assert np.allclose(s * s + c * c, 1.0)
    s0 = 0.5 / 40
    assert abs(E[0, 3] - math.sin(2 * math.pi * s0)) < 1e-15
    r = (np.repeat(np.arange(30), 40) + 0.5) / 30
    assert np.allclose(E[:, 11], 2 * r - 1)
    assert np.allclose(E[:, 12], np.sin(math.pi * r))
    X, P = ref.features(np.tile(workloads.conservative(1.0, 6.0, 0.0, 1.0, 2), (8 * 6, 1)), 8, 6, 40, 30,
                        (12.5, 0.01, 0.3, 1.0, 6.0, 1.0, 1.0, 0), rows=1216)
    assert X.shape == (1216, 32) and np.all(X[1200:] == 0) and np.all(X[:, 22:] == 0)
    assert np.allclose(P, [0.0, 1.0, 0.0, 0.0], atol=1e-14)
