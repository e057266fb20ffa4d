"""Parity of the warm-start kernels (include/ugkwp_mlp.h) with the FP64
reference oracle/warmstart_ref.py, through the C ABI.

BF16 operands are made exactly representable first, so both sides multiply
the same numbers; the kernels accumulate in FP32, so floating-point results
are compared within the FP32 accumulation bound
    |C - C_ref| <= 1e-5 * sum_k |A_ik B_jk|  (K <= 1024 terms of rounding 2^-24)
and BF16 outputs within one BF16 unit in the last place of the FP64 value."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import warmstart_ref as ref
import workloads

pytestmark = pytest.mark.gpu


def lib():
    from paper_2607_09552_amd import load_library
    return load_library()


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def vp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def bits(x):
    """BF16 bit patterns (int16) of values exactly representable in BF16."""
    x = np.asarray(x, dtype=np.float64)
    assert np.array_equal(ref.bf16(x), x)
    return (np.asarray(x, np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def vals(b):
    b = np.asarray(b).view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def within_bf16_ulp(got16, want64, abs_tol=0.0):
    """BF16 results within one unit in the last place of the FP64 values, plus
    abs_tol: the error the FP32 value had before rounding (cancellation makes
    it large relative to small results)."""
    got = vals(got16)
    ulp = np.abs(want64) * 2.0 ** -7
    return np.all(np.abs(got - want64) <= ulp + abs_tol)


@pytest.mark.parametrize("M,N,K,act", [(96, 64, 48, 1), (32, 256, 256, 1), (160, 32, 256, 0)])
def test_layer_forward(M, N, K, act):
    import torch
    g = np.random.default_rng(M + N + K)
    A = ref.bf16(g.standard_normal((M, K)))
    B = ref.bf16(g.standard_normal((N, K)) / math.sqrt(K))
    bias = g.standard_normal(N).astype(np.float32).astype(np.float64)
    Z = torch.empty((M, N), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(Z)
    Y16 = torch.empty((M, N), dtype=torch.int16, device="cuda")
    YT16 = torch.empty((N, M), dtype=torch.int16, device="cuda")
    dA, dB, db = dev(bits(A)), dev(bits(B)), dev(bias, torch.float32)
    rc = lib().ugkwp_mlp_layer(vp(dA), vp(dB), vp(db), M, N, K, act, vp(Z), vp(Y), vp(Y16), vp(YT16), None)
    assert rc == 0
    Zr = A @ B.T + bias
    Yr = ref.gelu(Zr) if act else Zr
    bound = 1e-5 * (np.abs(A) @ np.abs(B).T + np.abs(bias))
    assert np.all(np.abs(host(Z) - Zr) <= bound)
    assert np.all(np.abs(host(Y) - Yr) <= bound + 1e-6 * np.abs(Yr) + 1e-7)
    y16 = host(Y16)
    # the BF16 copy is the rounding of the FP32 result, and its transpose
    assert np.array_equal(vals(y16), ref.bf16(host(Y)))
    assert np.array_equal(host(YT16), y16.T)
    assert within_bf16_ulp(y16, Yr, abs_tol=1.2 * bound + 1e-7)


def test_layer_rejects_bad_shapes():
    import torch
    a = torch.zeros(64 * 32, dtype=torch.int16, device="cuda")
    L = lib()
    assert L.ugkwp_mlp_layer(vp(a), vp(a), None, 33, 32, 16, 0, None, None, None, None, None) == -1
    assert L.ugkwp_mlp_layer(vp(a), vp(a), None, 32, 32, 24, 0, None, None, None, None, None) == -1
    assert L.ugkwp_mlp_gemm_acc(vp(a), vp(a), 32, 32, 32, 8, vp(a), None) == -1


@pytest.mark.parametrize("K,kc", [(1008, 256), (4096, 512), (64, 1024)])
def test_gemm_acc_split_k(K, kc):
    import torch
    g = np.random.default_rng(K)
    M, N = 64, 96
    A = ref.bf16(g.standard_normal((M, K)))
    B = ref.bf16(g.standard_normal((N, K)))
    G0 = g.standard_normal((M, N)).astype(np.float32)
    G = dev(G0)
    dA, dB = dev(bits(A)), dev(bits(B))  # held until the kernel has run
    assert lib().ugkwp_mlp_gemm_acc(vp(dA), vp(dB), M, N, K, kc, vp(G), None) == 0
    want = G0 + A @ B.T
    bound = 1e-5 * (np.abs(A) @ np.abs(B).T) * (K / 256 + 1) + 1e-6 * np.abs(G0)
    assert np.all(np.abs(host(G) - want) <= bound)


@pytest.mark.parametrize("act", [1, 0])
def test_act_backward(act):
    import torch
    g = np.random.default_rng(7 + act)
    M, N = 200, 64  # M not a multiple of 64: columns straddle wavefronts
    dY = g.standard_normal((M, N)).astype(np.float32).astype(np.float64)
    Z = (2 * g.standard_normal((M, N))).astype(np.float32).astype(np.float64)
    dZ16 = torch.empty((M, N), dtype=torch.int16, device="cuda")
    dZT16 = torch.empty((N, M), dtype=torch.int16, device="cuda")
    db = torch.zeros(N, dtype=torch.float32, device="cuda")
    ddY, dZ = dev(dY, torch.float32), dev(Z, torch.float32)
    rc = lib().ugkwp_mlp_act_backward(vp(ddY), vp(dZ), M, N, act, vp(dZ16), vp(dZT16), vp(db), None)
    assert rc == 0
    want = dY * ref.gelu_grad(Z) if act else dY
    d16 = host(dZ16)
    if act:
        # FP32 erf and exp: GELU' within 1e-6 absolute (it has a root near -0.75)
        assert within_bf16_ulp(d16, want, abs_tol=1e-6 * np.abs(dY))
    else:
        assert np.array_equal(vals(d16), ref.bf16(dY))
    assert np.array_equal(host(dZT16), d16.T)
    assert np.allclose(host(db), want.sum(0), rtol=1e-5, atol=1e-5 * np.abs(want).sum(0).max())


def test_adam_and_bf16_copies():
    import torch
    g = np.random.default_rng(11)
    R, Cc = 64, 96
    w = g.standard_normal((R, Cc)).astype(np.float32).astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    dw, dm, dv = dev(w, torch.float32), dev(m, torch.float32), dev(v, torch.float32)
    w16 = torch.empty((R, Cc), dtype=torch.int16, device="cuda")
    wT16 = torch.empty((Cc, R), dtype=torch.int16, device="cuda")
    L = lib()
    for t in range(1, 4):
        gr = g.standard_normal((R, Cc)).astype(np.float32).astype(np.float64)
        dg = dev(gr, torch.float32)
        assert L.ugkwp_mlp_adam(vp(dw), vp(dm), vp(dv), vp(dg), R * Cc, Cc, 1e-2, 0.9, 0.999,
                                1e-8, t, vp(w16), vp(wT16), None) == 0
        w, m, v = ref.adam(w, m, v, gr, t, lr=1e-2)
        got = host(dw)
        assert np.allclose(got, w, rtol=2e-6, atol=2e-7)
        w = got.astype(np.float64)  # continue from the device's FP32 state
        m, v = host(dm).astype(np.float64), host(dv).astype(np.float64)
    assert np.array_equal(vals(host(w16)), ref.bf16(w))
    assert np.array_equal(host(wT16), host(w16).T)
    assert L.ugkwp_mlp_to_bf16(vp(dw), R * Cc, Cc, vp(w16), vp(wT16), None) == 0
    assert np.array_equal(vals(host(w16)), ref.bf16(w)) and np.array_equal(host(wT16), host(w16).T)


def test_mse_grad():
    import torch
    g = np.random.default_rng(5)
    M, N, n_out = 96, 32, 4
    Y = g.standard_normal((M, N)).astype(np.float32).astype(np.float64)
    T = g.standard_normal((M, n_out)).astype(np.float32).astype(np.float64)
    dY = torch.empty((M, N), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dYin, dT = dev(Y, torch.float32), dev(T, torch.float32)
    assert lib().ugkwp_mlp_mse_grad(vp(dYin), vp(dT), M, N, n_out, 2.0 / (M * n_out), vp(dY), vp(loss), None) == 0
    lr_, gr = ref.mse(Y, T, n_out)
    assert np.allclose(host(dY), gr, rtol=1e-6, atol=1e-9)
    assert abs(host(loss)[0] / (M * n_out) - lr_) <= 1e-5 * lr_


def _mlp_ref_params(mlp):
    return [(w.astype(np.float64), b.astype(np.float64)) for w, b in
            ((mlp.W[l].cpu().numpy(), mlp.b[l].cpu().numpy()) for l in range(len(mlp.W)))]


def test_training_step_gradients_and_update():
    """One step of the full 32-256-256-256-32 network: gradients against the
    FP64 reference with BF16 rounding at the kernels' points, then Adam."""
    import torch
    from paper_2607_09552_amd.warmstart import MLP
    g = np.random.default_rng(21)
    M = 256
    X = ref.bf16(g.standard_normal((M, 32)))
    T = g.standard_normal((M, 4)).astype(np.float32).astype(np.float64)
    mlp = MLP(seed=3)
    mlp.b = [b + torch.tensor(0.1 * g.standard_normal(b.shape[0]), dtype=torch.float32, device="cuda")
             for b in mlp.b]
    params = _mlp_ref_params(mlp)
    xb, xt, tt = dev(bits(X)), dev(np.ascontiguousarray(bits(X).T)), dev(T, torch.float32)
    mlp.train_step(xb, xt, tt, M, lr=0.0)
    Y, cache = ref.forward(params, X, q=ref.bf16)
    _, dY = ref.mse(Y, T, 4)
    grads, _ = ref.backward(params, cache, dY, q=ref.bf16)
    torch.cuda.synchronize()
    for l, (gw, gb) in enumerate(grads):
        got_w, got_b = mlp.gW[l].cpu().numpy(), mlp.gb[l].cpu().numpy()
        assert np.linalg.norm(got_w - gw) <= 2e-3 * np.linalg.norm(gw), l
        assert np.linalg.norm(got_b - gb) <= 2e-3 * np.linalg.norm(gb), l
    # lr = 0 left the weights; a real step is Adam on the device gradients
    assert all(np.array_equal(mlp.W[l].cpu().numpy(), params[l][0].astype(np.float32)) for l in range(4))
    gws = [mlp.gW[l].cpu().numpy().astype(np.float64) for l in range(4)]
    mlp.train_step(xb, xt, tt, M, lr=1e-3)
    torch.cuda.synchronize()
    # t = 2 moments from two gradients: the first (gws) and the second (same
    # weights, same batch: the same gradient up to accumulation order)
    for l in range(4):
        g2 = mlp.gW[l].cpu().numpy().astype(np.float64)
        m1 = 0.1 * gws[l]
        v1 = 0.001 * gws[l] ** 2
        w, _, _ = ref.adam(params[l][0], m1, v1, g2, 2, lr=1e-3)
        assert np.allclose(mlp.W[l].cpu().numpy(), w, rtol=1e-5, atol=1e-6), l


def test_training_reduces_the_loss():
    import torch
    from paper_2607_09552_amd.warmstart import MLP
    g = np.random.default_rng(8)
    M = 1024
    X = ref.bf16(np.concatenate([g.uniform(-1, 1, (M, 4)), np.zeros((M, 28))], axis=1))
    T = np.stack([np.sin(3 * X[:, 0]), X[:, 1] * X[:, 2], np.cos(2 * X[:, 3]), X[:, 0] ** 2], axis=1)
    mlp = MLP(seed=1)
    xb, xt, tt = dev(bits(X)), dev(np.ascontiguousarray(bits(X).T)), dev(T, torch.float32)
    first = None
    for it in range(300):
        loss = mlp.train_step(xb, xt, tt, M, lr=2e-3)
        if it == 0:
            first = float(loss.item())
    last = float(loss.item())
    assert last < 0.02 * first, (first, last)


def _smooth_coarse(nct, ncr, Ma):
    """A smooth, positive coarse state (not a solution) for the feature map."""
    i = np.tile(np.arange(nct), ncr)
    j = np.repeat(np.arange(ncr), nct)
    th = 2 * np.pi * i / nct
    rho = 1.0 + 2.0 * np.exp(-j / 5.0) * (1 + np.cos(th)) / 2
    U = Ma * math.sqrt(5.0 / 3.0)
    ux = U * (1 - np.exp(-j / 4.0)) * np.cos(0.3 * th)
    uy = U * 0.2 * np.sin(th) * np.exp(-j / 6.0)
    T = 1.0 + 30.0 * np.exp(-j / 3.0)
    return workloads.conservative(rho, ux, uy, T, 2)


@pytest.mark.parametrize("nct,ncr,nft,nfr", [(40, 30, 200, 150), (8, 6, 40, 30)])
def test_features_and_decode(nct, ncr, nft, nfr):
    import torch
    from paper_2607_09552_amd import WsCase
    Ma, Kn, Tw = 14.0, 0.02, 0.25
    U = Ma * math.sqrt(5.0 / 3.0)
    Wc = _smooth_coarse(nct, ncr, Ma)
    nf = nft * nfr
    rows = nf + (-nf) % 32 + 32
    case = WsCase(Ma=Ma, Kn=Kn, Tw=Tw, rho_inf=1.0, U_inf=U, T_inf=1.0, R=1.0, D=0)
    X16 = torch.full((rows, 32), 7, dtype=torch.int16, device="cuda")
    XT16 = torch.empty((32, rows), dtype=torch.int16, device="cuda")
    P32 = torch.empty((nf, 4), dtype=torch.float32, device="cuda")
    L = lib()
    dWc = dev(Wc)
    assert L.ugkwp_ws_features(vp(dWc), nct, ncr, nft, nfr, C.byref(case), rows, vp(X16), vp(XT16), vp(P32),
                               None) == 0
    Xr, Pr = ref.features(Wc, nct, ncr, nft, nfr, (Ma, Kn, Tw, 1.0, U, 1.0, 1.0, 0), rows=rows)
    x16 = host(X16)
    assert np.all(x16[nf:] == 0)
    assert np.array_equal(host(XT16), x16.T)
    # BF16 of the FP32 rounding of the FP64 value: within one BF16 ulp (zeros exact)
    assert within_bf16_ulp(x16[:nf], Xr[:nf], abs_tol=1e-7)
    assert np.allclose(host(P32), Pr, rtol=1e-6, atol=1e-6)
    # decode of a correction
    g = np.random.default_rng(3)
    Y = (0.1 * g.standard_normal((nf, 32))).astype(np.float32)
    W = torch.empty((nf, 4), dtype=torch.float64, device="cuda")
    dY = dev(Y)
    assert L.ugkwp_ws_decode(vp(dY), 32, vp(P32), nf, C.byref(case), vp(W), None) == 0
    want = ref.decode(Y.astype(np.float64), host(P32).astype(np.float64), 1.0, U, 1.0)
    assert np.allclose(host(W), want, rtol=1e-13, atol=1e-13)
    bad = WsCase(Ma=Ma, Kn=-1.0, Tw=Tw, rho_inf=1.0, U_inf=U, T_inf=1.0, R=1.0, D=0)
    assert L.ugkwp_ws_features(vp(dWc), nct, ncr, nft, nfr, C.byref(bad), rows, vp(X16), None, None, None) == -1
    assert L.ugkwp_ws_features(vp(dWc), nct, ncr, nft, nfr, C.byref(case), nf - 1, vp(X16), None, None,
                               None) == -1


def test_fused_forward_matches_layers_and_reference():
    """The one-kernel forward (activations in registers, permuted K order)
    against the per-layer kernels and the FP64 reference with BF16 rounding
    of the activations."""
    import torch
    from paper_2607_09552_amd.warmstart import MLP
    g = np.random.default_rng(31)
    M = 96
    X = ref.bf16(g.standard_normal((M, 32)))
    mlp = MLP(seed=5)
    mlp.b = [b + torch.tensor(0.1 * g.standard_normal(b.shape[0]), dtype=torch.float32, device="cuda")
             for b in mlp.b]
    xb = dev(bits(X))
    Yf = host(mlp.infer(xb, M)).astype(np.float64)
    Yl = host(mlp.forward(xb, M)).astype(np.float64)
    Yr, _ = ref.forward(_mlp_ref_params(mlp), X, q=ref.bf16)
    scale = np.abs(Yr).max()
    # FP32 accumulation in another order can flip an activation's BF16
    # rounding: differences stay at that level
    assert np.max(np.abs(Yf - Yr)) <= 2e-2 * scale
    assert np.max(np.abs(Yf - Yl)) <= 2e-2 * scale
    assert np.median(np.abs(Yf - Yr)) <= 1e-4 * scale
    # packing: layer 1's fragments are the BF16 weights in the permuted order
    Wf = host(mlp.Wf[1]).reshape(-1, 64, 8)
    W1 = mlp.W[1].cpu().numpy().astype(np.float64)
    S = W1.shape[1] // 16
    for t, s_, lane, e in ((0, 0, 0, 0), (3, 5, 37, 6), (7, 15, 63, 7), (2, 9, 31, 3)):
        h = lane // 32
        k = 16 * s_ + 8 * (e // 4) + 4 * h + e % 4
        assert vals(Wf[t * S + s_, lane, e]) == ref.bf16(W1[32 * t + lane % 32, k])
    L = lib()
    wd = (C.c_int32 * 5)(32, 256, 128, 256, 32)
    wp = (C.c_void_p * 4)(*[w.data_ptr() for w in mlp.Wf])
    bp = (C.c_void_p * 4)(*[b.data_ptr() for b in mlp.b])
    Y = torch.empty((M, 32), dtype=torch.float32, device="cuda")
    assert L.ugkwp_mlp_forward(vp(xb), M, 4, wd, wp, bp, vp(Y), None) == -1
    wd[2] = 256
    assert L.ugkwp_mlp_forward(vp(xb), M - 1, 4, wd, wp, bp, vp(Y), None) == -1


def test_warm_start_end_to_end_and_batched_command(tmp_path):
    """The whole warm start (coarse wave-particle solve, features, fused
    network, decode) gives a valid fine field with a hot shock layer
    (stagnation temperature T_0 = T_inf (1 + Ma^2/3) = 76 at Ma 15) and a
    cold leeward side, which the fine solver takes as its initial state; the
    batched time-to-residual command runs both legs on two held-out cases
    (shortened) and reports every case."""
    import torch
    from paper_2607_09552_amd import warmstart as ws
    ws.use_own_stream()
    try:
        _warm_start_checks(ws, tmp_path)
    finally:
        torch.cuda.synchronize()
        torch.cuda.set_stream(torch.cuda.default_stream())


def _warm_start_checks(ws, tmp_path):
    import json
    from paper_2607_09552_amd import Solver
    wl = ws.fine_case(15.0, 0.01, 0.2, n_ref=20)
    W0, info = ws.warm_start(15.0, 0.01, 0.2, wl=wl)
    nf = ws.FINE[0] * ws.FINE[1]
    assert W0.shape == (nf, 4) and np.all(np.isfinite(W0))
    rho = W0[:, 0]
    T = (W0[:, 3] - 0.5 * (W0[:, 1] ** 2 + W0[:, 2] ** 2) / rho) / (1.5 * rho)
    assert np.all(rho > 0) and np.all(T > 0)
    assert T.max() > 20.0 and T.min() < 1.0, (T.min(), T.max())
    assert info["seconds"] > info["coarse_seconds"] > 0
    s = Solver(wl, W0=W0, precision="mixed")
    s.step(20)
    assert np.all(np.isfinite(s.fields())) and s.residual()[2] == 20
    s.close()
    out = tmp_path / "batched.json"
    ws.main(["batched", "--n-cases", "2", "--n-ref", "20", "--max-steps", "120", "--chunk", "60",
             "--legs", "f64,batch-warm", "--out", str(out)])
    r = json.loads(out.read_text())
    assert [c["steps"] for c in r["f64"]["cases"]] == [120, 120]
    assert r["batch-warm"]["steps"] == 120 and len(r["batch-warm"]["case_r_avg"]) == 2
    assert r["batch-warm"]["warm_start_seconds"] > 0 and np.all(np.isfinite(r["batch-warm"]["case_r_avg"]))


def test_network_beats_the_upsampled_coarse_field_on_held_out_draws():
    """What the trained network gains: for the first three held-out draws
    (never trained on), the fine solve's steady field (200 x 150, N_ref 100,
    mixed precision, mean over 4000 steps after 4000 as for the training
    targets, seeds of their own) is
    computed here, and the network's field must be closer to it than the
    bilinearly upsampled coarse field it starts from: RMS error of every
    normalized primitive (ln rho, u/U, v/U, ln T) smaller on every draw, and
    on average at most half the upsampled error.  Untrained or wrongly
    applied weights (a correction with the wrong sign, outputs in another
    order) fail it."""
    import torch
    from paper_2607_09552_amd import warmstart as ws
    ws.use_own_stream()
    try:
        _network_gain_checks(ws)
    finally:
        torch.cuda.synchronize()
        torch.cuda.set_stream(torch.cuda.default_stream())


def _network_gain_checks(ws):
    import torch
    from paper_2607_09552_amd import Solver
    cases = [tuple(c) for c in ws.draws(16, 4)[:3]]
    Wc, _ = ws.coarse_solve(cases)
    wls = [ws.fine_case(*c, n_ref=100, seed=7000 + k) for k, c in enumerate(cases)]
    s = Solver.batch(wls, stream=ws._stream().value, precision="mixed", tuned=False)
    try:
        Wm = ws.averaged_fields(s, 4000, 4000, 10).cpu().numpy()
        ranges = [s.case_range(k)[:2] for k in range(len(cases))]
    finally:
        s.close()
    mlp = ws.MLP.load()
    nf = ws.FINE[0] * ws.FINE[1]
    rows = nf + (-nf) % 32
    e_up, e_nn = [], []
    for k, c in enumerate(cases):
        c0, n = ranges[k]
        target = ws._norm_prim(Wm[c0:c0 + n], wls[k])
        X16, _, P32 = ws.features(Wc[k], ws.ws_case(wls[k], *c), rows, XT=False)
        Y = mlp.infer(X16, rows)[:nf, :4].float().cpu().numpy()
        P = P32.cpu().numpy().astype(np.float64)
        e_up.append(np.sqrt(np.mean((target - P) ** 2, axis=0)))
        e_nn.append(np.sqrt(np.mean((target - P - Y) ** 2, axis=0)))
    e_up, e_nn = np.array(e_up), np.array(e_nn)
    assert np.all(e_nn < e_up), (e_up, e_nn)
    assert np.all(e_nn.mean(0) < 0.5 * e_up.mean(0)), (e_up.mean(0), e_nn.mean(0))
