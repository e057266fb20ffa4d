"""Learned warm start of steady cylinder runs.

The method fixes the local time steps from the initial field and marches to
a steady state (Sec. IV, Eq. (33); the test cases of Sec. V start from the
free stream).  A better initial field shortens the march.  This module
predicts one:

  1. a coarse UGKWP-LTS solve of the same case on a 40 x 30 O-grid whose
     nodes are every fifth node of the fine 200 x 150 grid (50 particles per
     cell), its fields averaged over a window after a fixed transient.  (The
     wave-only mode, i.e. the gas-kinetic scheme without particles, cannot
     carry these starts: gas leaving the leeward wall faster than the escape
     speed 2c/(gamma - 1) = 3c opens a vacuum, and the blow-up follows.);
  2. features per fine cell (ugkwp_ws_features): the coarse normalized
     primitives interpolated bilinearly in cell-index space, the case
     parameters (Ma, Kn, T_w) and a Fourier encoding of the cell indices;
  3. a multilayer perceptron (32 -> 256 -> 256 -> 256 -> 32, GELU) whose
     first four outputs correct the interpolated primitives
     (ugkwp_ws_decode turns them into the conservative initial field).

Training fits the corrections to time-averaged steady fields of full UGKWP
runs of sampled cases (mean squared error, Adam).  Every arithmetic step of
inference and training runs in the library's kernels (dense layers on the
BF16 matrix cores); torch only holds device memory and clears gradient
buffers.  Data preparation (the time averages of the solver's fields that
become the targets and the coarse input, the held-out error figures) is
host numpy.

Command line (GPU): ``python -m paper_2607_09552_amd.warmstart data|train|eval``.
"""
from __future__ import annotations

import argparse
import contextlib
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

from . import Solver, UgkwpError, WsCase, load_library

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
WEIGHTS = os.path.join(HERE, "warmstart_weights.npz")
WIDTHS = (32, 256, 256, 256, 32)
N_OUT = 4
FINE = (200, 150)
COARSE = (40, 30)
# ranges of the sampled cases
MA_RANGE, KN_RANGE, TW_RANGE = (5.0, 20.0), (0.005, 0.2), (0.1, 0.5)
# coarse solve: particles per cell, steps before and during averaging
COARSE_NREF, COARSE_TRANSIENT, COARSE_AVERAGE, COARSE_EVERY = 50, 1500, 1500, 5


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _chk(rc, what):
    if rc != 0:
        raise UgkwpError(rc, what)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@contextlib.contextmanager
def _nonnull_stream():
    """Run the body on a real stream: a solver given the null stream runs on
    its own non-blocking one, unordered with torch's null-stream work."""
    import torch
    if torch.cuda.current_stream().cuda_stream != 0:
        yield
        return
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        yield
    torch.cuda.current_stream().wait_stream(st)


def use_own_stream():
    """Make a fresh (default-priority) stream torch's current one, so that the
    solver, these kernels and torch's own work are ordered on one stream."""
    import torch
    torch.cuda.set_device(0)
    torch.cuda.set_stream(torch.cuda.Stream())


def draws(n, seed):
    """n cases (Ma, Kn, T_w): Ma and T_w uniform, Kn log-uniform over the
    ranges above (numpy generator seeded with `seed`)."""
    u = np.random.default_rng(seed).random((n, 3))
    ma = MA_RANGE[0] + (MA_RANGE[1] - MA_RANGE[0]) * u[:, 0]
    kn = KN_RANGE[0] * (KN_RANGE[1] / KN_RANGE[0]) ** u[:, 1]
    tw = TW_RANGE[0] + (TW_RANGE[1] - TW_RANGE[0]) * u[:, 2]
    return np.stack([ma, kn, tw], axis=1)


def fine_case(Ma, Kn, Tw, n_ref=400, seed=1):
    import workloads
    return workloads.cylinder(n_theta=FINE[0], n_r=FINE[1], Ma=Ma, Kn=Kn, Tw=Tw, n_ref=n_ref, seed=seed)


def coarse_case(Ma, Kn, Tw, n_ref=COARSE_NREF, seed=3):
    """The case on the O-grid made of every fifth fine node: same outer
    radius, first cell height the sum of the first five fine ones."""
    import workloads
    f = workloads.ogrid(FINE[0], FINE[1])[3]
    rt, rr = FINE[0] // COARSE[0], FINE[1] // COARSE[1]
    h1 = 1e-4 * (f ** rr - 1.0) / (f - 1.0)
    assert rt * COARSE[0] == FINE[0] and rr * COARSE[1] == FINE[1]
    return workloads.cylinder(n_theta=COARSE[0], n_r=COARSE[1], h1=h1, Ma=Ma, Kn=Kn, Tw=Tw, n_ref=n_ref, seed=seed)


def ws_case(wl, Ma, Kn, Tw):
    """Warm-start case record of workload wl (its free stream and gas)."""
    g, r = wl["gas"], wl["ref"]
    return WsCase(Ma=Ma, Kn=Kn, Tw=Tw, rho_inf=r["rho_inf"], U_inf=math.hypot(*r["u_inf"]), T_inf=r["T_inf"],
                  R=g["R"], D=g["D"])


def cylinder_ws_case(Ma, Kn, Tw):
    """Warm-start case record of the cylinder workload (rho_inf = T_inf = R = 1,
    U_inf = Ma sqrt(5/3), monatomic) without building its mesh."""
    import workloads
    return WsCase(Ma=Ma, Kn=Kn, Tw=Tw, rho_inf=1.0, U_inf=Ma * math.sqrt(workloads.GAMMA_MONATOMIC), T_inf=1.0,
                  R=1.0, D=0)


def averaged_fields(s, transient, average, every, log=None):
    """Mean of the conservative fields of solver s over `average` steps
    (sampled every `every`) after `transient` steps, summed on the host
    (data preparation, not the network's arithmetic) and returned as a
    device tensor for the feature kernel."""
    import torch
    s.step(transient)
    acc = np.zeros((s.nc, s.nw), dtype=np.float64)
    n = max(1, average // every)
    for k in range(n):
        s.step(every)
        acc += s.fields()
        if log and (k + 1) % max(1, n // 4) == 0:
            log(f"averaged {(k + 1) * every} steps")
    return torch.tensor(acc / n, device="cuda")


def coarse_solve(cases, transient=COARSE_TRANSIENT, average=COARSE_AVERAGE, every=COARSE_EVERY):
    """Coarse solves of cases [(Ma, Kn, T_w)] in one batch; returns (device
    mean fields [n_case, ncr nct, 4] FP64, seconds)."""
    import torch
    wls = [coarse_case(*c, seed=3000 + k) for k, c in enumerate(cases)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with _nonnull_stream():
        s = Solver.batch(wls, stream=_stream().value, precision="mixed", tuned=False)
        try:
            W = averaged_fields(s, transient, average, every)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            s.close()
    return W.view(len(cases), COARSE[0] * COARSE[1], 4), dt


def _bf16_buf(*shape):
    import torch
    return torch.empty(shape, dtype=torch.int16, device="cuda")


class MLP:
    """FP32 master weights W_l [out x in], b_l [out]; BF16 copies W_l and
    W_l^T for the matrix-core layers; Adam moments."""

    def __init__(self, widths=WIDTHS, seed=0, weights=None):
        import torch
        load_library()
        self.widths = tuple(widths)
        rng = np.random.default_rng(seed)
        self.W, self.b = [], []
        for l, (i, o) in enumerate(zip(widths[:-1], widths[1:])):
            if weights is not None:
                w, b = weights[f"W{l}"], weights[f"b{l}"]
            else:
                scale = math.sqrt(2.0 / i) * (0.1 if l == len(widths) - 2 else 1.0)
                w, b = rng.standard_normal((o, i)) * scale, np.zeros(o)
            self.W.append(torch.tensor(np.asarray(w, np.float32), device="cuda").contiguous())
            self.b.append(torch.tensor(np.asarray(b, np.float32), device="cuda").contiguous())
        self.W16 = [_bf16_buf(*w.shape) for w in self.W]
        self.WT16 = [_bf16_buf(w.shape[1], w.shape[0]) for w in self.W]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.gW = [torch.zeros_like(w) for w in self.W]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.t = 0
        self._bufs = {}
        self._packed_at = None
        self.Wf = [_bf16_buf(w.numel()) for w in self.W]
        self._sync_bf16()

    def _sync_bf16(self):
        L, st = load_library(), _stream()
        for w, w16, wt16 in zip(self.W, self.W16, self.WT16):
            _chk(L.ugkwp_mlp_to_bf16(_vp(w), w.numel(), w.shape[1], _vp(w16), _vp(wt16), st), "to_bf16")

    def weights(self):
        out = {}
        for l, (w, b) in enumerate(zip(self.W, self.b)):
            out[f"W{l}"] = w.detach().cpu().numpy()
            out[f"b{l}"] = b.detach().cpu().numpy()
        return out

    def save(self, path, meta=None):
        np.savez(path, **self.weights(), meta=json.dumps(meta or {}))

    @classmethod
    def load(cls, path=WEIGHTS):
        z = np.load(path)
        ws = {k: z[k] for k in z.files if k != "meta"}
        n = len([k for k in ws if k.startswith("W")])
        widths = [ws["W0"].shape[1]] + [ws[f"W{l}"].shape[0] for l in range(n)]
        return cls(widths=widths, weights=ws)

    def _buffers(self, M):
        import torch
        if M in self._bufs:
            return self._bufs[M]
        wd = self.widths
        nl = len(wd) - 1
        b = dict(
            H16=[None] + [_bf16_buf(M, wd[l]) for l in range(1, nl)],
            HT16=[None] + [_bf16_buf(wd[l], M) for l in range(1, nl)],
            Z=[torch.empty((M, wd[l + 1]), dtype=torch.float32, device="cuda") for l in range(nl)],
            Y=torch.empty((M, wd[-1]), dtype=torch.float32, device="cuda"),
            dY=torch.empty((M, max(wd)), dtype=torch.float32, device="cuda"),
            dH=torch.empty((M, max(wd)), dtype=torch.float32, device="cuda"),
            dZ16=_bf16_buf(M * max(wd)),
            dZT16=_bf16_buf(M * max(wd)),
            loss=torch.zeros(1, dtype=torch.float32, device="cuda"),
        )
        self._bufs = {M: b}  # one batch size at a time
        return b

    def fused_ok(self):
        return self.widths == WIDTHS

    def infer(self, X16, M):
        """Network output [M x 32] FP32 for BF16 features X16 [M x 32], in one
        kernel (activations in registers); the per-layer path for other
        widths."""
        import torch
        if not self.fused_ok():
            return self.forward(X16, M)
        L, st = load_library(), _stream()
        if self._packed_at != self.t:
            for l, w in enumerate(self.W):
                _chk(L.ugkwp_mlp_pack(_vp(w), w.shape[0], w.shape[1], 0 if l == 0 else 1, _vp(self.Wf[l]), st),
                     "pack")
            self._packed_at = self.t
        Y = torch.empty((M, self.widths[-1]), dtype=torch.float32, device="cuda")
        nl = len(self.widths) - 1
        wd = (C.c_int32 * (nl + 1))(*self.widths)
        wp = (C.c_void_p * nl)(*[w.data_ptr() for w in self.Wf])
        bp = (C.c_void_p * nl)(*[b.data_ptr() for b in self.b])
        _chk(L.ugkwp_mlp_forward(_vp(X16), M, nl, wd, wp, bp, _vp(Y), st), "forward")
        return Y

    def forward(self, X16, M, train=False):
        """Network output [M x 32] FP32 for BF16 features X16 [M x 32], one
        launch per layer (train: keep what the backward pass needs)."""
        L, st = load_library(), _stream()
        b = self._buffers(M)
        nl = len(self.widths) - 1
        H = X16
        for l in range(nl):
            last = l == nl - 1
            _chk(L.ugkwp_mlp_layer(_vp(H), _vp(self.W16[l]), _vp(self.b[l]), M, self.widths[l + 1], self.widths[l],
                                   0 if last else 1, _vp(b["Z"][l]) if (train and not last) else None,
                                   _vp(b["Y"]) if last else None, None if last else _vp(b["H16"][l + 1]),
                                   _vp(b["HT16"][l + 1]) if (train and not last) else None, st), "layer")
            if not last:
                H = b["H16"][l + 1]
        return b["Y"]

    def train_step(self, X16, XT16, T, M, lr, beta1=0.9, beta2=0.999, eps=1e-8, k_chunk=512, want_loss=True):
        """One Adam step on the mean squared error of the first four outputs
        against T [M x 4]; returns the device loss (sum of squares), or None
        without want_loss."""
        L, st = load_library(), _stream()
        wd = self.widths
        nl = len(wd) - 1
        b = self._buffers(M)
        Y = self.forward(X16, M, train=True)
        if want_loss:
            b["loss"].zero_()
        dY = b["dY"]
        _chk(L.ugkwp_mlp_mse_grad(_vp(Y), _vp(T), M, wd[-1], N_OUT, 2.0 / (M * N_OUT), _vp(dY),
                                  _vp(b["loss"]) if want_loss else None, st), "mse_grad")
        for g in self.gW + self.gb:
            g.zero_()
        G = dY  # gradient w.r.t. the current layer's output, [M x out]
        for l in range(nl - 1, -1, -1):
            o, i = wd[l + 1], wd[l]
            Hin, HinT = (X16, XT16) if l == 0 else (b["H16"][l], b["HT16"][l])
            _chk(L.ugkwp_mlp_act_backward(_vp(G), _vp(b["Z"][l]) if l < nl - 1 else None, M, o,
                                          1 if l < nl - 1 else 0, _vp(b["dZ16"]), _vp(b["dZT16"]), _vp(self.gb[l]),
                                          st), "act_backward")
            _chk(L.ugkwp_mlp_gemm_acc(_vp(b["dZT16"]), _vp(HinT), o, i, M, k_chunk, _vp(self.gW[l]), st),
                 "gemm_acc")
            if l > 0:
                dH = b["dH"] if G.data_ptr() != b["dH"].data_ptr() else b["dY"]
                _chk(L.ugkwp_mlp_layer(_vp(b["dZ16"]), _vp(self.WT16[l]), None, M, i, o, 0, None, _vp(dH), None,
                                       None, st), "layer_backward")
                G = dH
        self.t += 1
        for l in range(nl):
            w = self.W[l]
            _chk(L.ugkwp_mlp_adam(_vp(w), _vp(self.mW[l]), _vp(self.vW[l]), _vp(self.gW[l]), w.numel(), w.shape[1],
                                  lr, beta1, beta2, eps, self.t, _vp(self.W16[l]), _vp(self.WT16[l]), st), "adam")
            bb = self.b[l]
            _chk(L.ugkwp_mlp_adam(_vp(bb), _vp(self.mb[l]), _vp(self.vb[l]), _vp(self.gb[l]), bb.numel(), bb.numel(),
                                  lr, beta1, beta2, eps, self.t, None, None, st), "adam")
        return b["loss"] if want_loss else None


def features(Wc, case, rows, XT=True):
    """Device features of the fine grid for one case from its coarse fields
    Wc (device [ncr nct, 4] FP64): (X16 [rows x 32], XT16 or None, P32)."""
    import torch
    L = load_library()
    nf = FINE[0] * FINE[1]
    X16 = _bf16_buf(rows, 32)
    XT16 = _bf16_buf(32, rows) if XT else None
    P32 = torch.empty((nf, 4), dtype=torch.float32, device="cuda")
    _chk(L.ugkwp_ws_features(_vp(Wc), COARSE[0], COARSE[1], FINE[0], FINE[1], C.byref(case), rows, _vp(X16),
                             _vp(XT16) if XT else None, _vp(P32), _stream()), "features")
    return X16, XT16, P32


def predict(mlp, Wc, case):
    """Fine initial field (host [nf x 4] FP64) for one case."""
    import torch
    L = load_library()
    nf = FINE[0] * FINE[1]
    rows = (nf + 31) // 32 * 32
    X16, _, P32 = features(Wc, case, rows, XT=False)
    Y = mlp.infer(X16, rows)
    W = torch.empty((nf, 4), dtype=torch.float64, device="cuda")
    _chk(L.ugkwp_ws_decode(_vp(Y), Y.shape[1], _vp(P32), nf, C.byref(case), _vp(W), _stream()), "decode")
    return W.cpu().numpy()


def warm_start(Ma, Kn, Tw, mlp=None, wl=None):
    """Initial field for the fine case (Ma, Kn, T_w): coarse wave-only solve,
    features, network, decode.  Returns (W0 [nf x 4] host, info)."""
    import torch
    mlp = mlp or MLP.load()
    t0 = time.perf_counter()
    Wc, tc = coarse_solve([(Ma, Kn, Tw)])
    W0 = predict(mlp, Wc[0], ws_case(wl or fine_case(Ma, Kn, Tw, n_ref=1), Ma, Kn, Tw))
    torch.cuda.synchronize()
    return W0, dict(coarse_seconds=tc, seconds=time.perf_counter() - t0)


def _norm_prim(W, wl):
    g, r = wl["gas"], wl["ref"]
    rho = W[:, 0]
    u, v = W[:, 1] / rho, W[:, 2] / rho
    T = (W[:, 3] / rho - 0.5 * (u * u + v * v)) / (0.5 * (3 + g["D"]) * g["R"])
    U = math.hypot(*r["u_inf"])
    return np.stack([np.log(rho / r["rho_inf"]), u / U, v / U, np.log(T / r["T_inf"])], axis=1)


# ---------------------------------------------------------------- command line


def cmd_data(a):
    """Steady fields of sampled cases: coarse wave-only solves and time-averaged
    fine UGKWP runs (mixed precision, n_ref particles per cell), in batches."""
    import torch
    use_own_stream()
    cases = np.concatenate([draws(a.n_train, a.train_seed), draws(a.n_test, 4)])
    n = len(cases)
    print(f"coarse solves: {n} cases", flush=True)
    Wc, dt = coarse_solve([tuple(c) for c in cases])
    print(f"  {dt:.1f} s", flush=True)
    nf = FINE[0] * FINE[1]
    P = np.zeros((n, nf, 4), dtype=np.float16)
    for b0 in range(0, n, a.batch):
        idx = list(range(b0, min(n, b0 + a.batch)))
        wls = [fine_case(*cases[k], n_ref=a.n_ref, seed=2000 + k) for k in idx]
        t0 = time.perf_counter()
        s = Solver.batch(wls, stream=_stream().value, precision="mixed", tuned=False)

        def log(msg):
            torch.cuda.synchronize()
            print(f"  cases {idx[0]}-{idx[-1]}: {msg} {time.perf_counter() - t0:.1f} s", flush=True)

        acc = averaged_fields(s, a.transient, a.average, a.every, log)
        Wm = acc.cpu().numpy()
        for j, k in enumerate(idx):
            c0, ncells = s.case_range(j)[:2]
            P[k] = _norm_prim(Wm[c0:c0 + ncells], wls[j]).astype(np.float16)
        s.close()
        del acc
        torch.cuda.empty_cache()
    np.savez(a.out, cases=cases, n_train=a.n_train, coarse=Wc.cpu().numpy(), fine=P, n_ref=a.n_ref,
             transient=a.transient, average=a.average, train_seed=a.train_seed)
    print(f"wrote {a.out}", flush=True)


def cmd_train(a):
    import torch
    use_own_stream()
    # one or more data files: the training cases of all, the held-out cases of
    # the first
    zs = [np.load(f) for f in a.data.split(",")]
    z = zs[0]
    parts = [(zz["cases"][: int(zz["n_train"])], zz["coarse"][: int(zz["n_train"])], zz["fine"][: int(zz["n_train"])])
             for zz in zs]
    ntr = sum(len(p[0]) for p in parts)
    n0 = int(z["n_train"])
    cases = np.concatenate([p[0] for p in parts] + [z["cases"][n0:]])
    coarse = torch.tensor(np.concatenate([p[1] for p in parts] + [z["coarse"][n0:]]), device="cuda")
    fine = np.concatenate([p[2] for p in parts] + [z["fine"][n0:]]).astype(np.float32)
    nf = FINE[0] * FINE[1]
    # assemble the features and the target corrections of every case
    Xs, XTs, Ts = [], [], []
    for k in range(len(cases)):
        c = cylinder_ws_case(*cases[k])
        X16, _, P32 = features(coarse[k], c, nf + (-nf) % 32, XT=False)
        Xs.append(X16[:nf].cpu().numpy())
        Ts.append(fine[k] - P32.cpu().numpy())
    X = np.stack(Xs)  # [n, nf, 32] int16 (BF16 bits)
    T = np.stack(Ts).astype(np.float32)
    Xtr, Ttr = X[:ntr].reshape(-1, 32), T[:ntr].reshape(-1, 4)
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(Xtr))
    M = a.batch
    nb = len(Xtr) // M
    Xb = Xtr[perm[: nb * M]].reshape(nb, M, 32)
    Tb = Ttr[perm[: nb * M]].reshape(nb, M, 4)
    Xd = torch.tensor(Xb, device="cuda")
    XTd = torch.tensor(np.ascontiguousarray(Xb.transpose(0, 2, 1)), device="cuda")
    Td = torch.tensor(Tb, device="cuda")
    mlp = MLP(seed=a.seed)
    print(f"training: {nb} batches of {M}, {a.steps} steps", flush=True)
    t0 = time.perf_counter()
    hist = []
    for it in range(a.steps):
        lr = a.lr * 0.5 * (1.0 + math.cos(math.pi * it / a.steps))
        j = it % nb
        log = (it + 1) % a.log_every == 0 or it == 0
        loss = mlp.train_step(Xd[j], XTd[j], Td[j], M, lr, want_loss=log)
        if log:
            v = float(loss.item()) / (M * N_OUT)
            hist.append((it + 1, v))
            print(f"  step {it + 1} loss {v:.4e} lr {lr:.2e} {time.perf_counter() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    # per-case errors: coarse upsample alone vs corrected
    def case_err(k):
        rows = nf + (-nf) % 32
        Xk = torch.tensor(np.concatenate([X[k], np.zeros((rows - nf, 32), np.int16)]), device="cuda")
        Y = mlp.infer(Xk, rows)[:nf, :4].cpu().numpy()
        e_up = np.sqrt(np.mean(T[k] ** 2, axis=0))
        e_nn = np.sqrt(np.mean((T[k] - Y) ** 2, axis=0))
        return e_up, e_nn

    rep = {}
    for name, ks in (("train", range(min(ntr, 16))), ("held_out", range(ntr, len(cases)))):
        eu, en = zip(*[case_err(k) for k in ks])
        rep[name] = dict(rms_upsampled=np.mean(eu, axis=0).tolist(), rms_network=np.mean(en, axis=0).tolist())
        print(f"  {name}: RMS error (ln rho, u, v, ln T) upsampled {np.round(rep[name]['rms_upsampled'], 4)} "
              f"network {np.round(rep[name]['rms_network'], 4)}", flush=True)
    meta = dict(steps=a.steps, batch=M, lr=a.lr, seconds=train_s, history=hist, errors=rep,
                data=dict(n_train=ntr, n_test=len(cases) - ntr, n_ref=int(z["n_ref"]), transient=int(z["transient"]),
                          average=int(z["average"]), files=a.data))
    mlp.save(a.out, meta)
    print(f"wrote {a.out} ({train_s:.1f} s)", flush=True)


def cmd_eval(a):
    """Time to residual (r_avg < target) from the free stream and from the
    warm start, same case, same precision."""
    import torch
    use_own_stream()
    mlp = MLP.load(a.weights)
    out = []
    cases = [(a.ma, a.kn, a.tw)] if a.ma else [tuple(c) for c in draws(a.n_test, 4)[a.skip: a.skip + a.n_cases]]
    n0, n1 = (int(x) for x in a.reference.split(",")) if a.reference else (0, 0)
    for (Ma, Kn, Tw) in cases:
        wl = fine_case(Ma, Kn, Tw, n_ref=a.n_ref, seed=1)
        # time steps from the freestream for every run (the reference and the
        # free-stream leg have them anyway): all runs share one steady state
        wl["dt_source"] = {"initial": 0, "freestream": 1}[a.dt_source]
        res = dict(Ma=Ma, Kn=Kn, Tw=Tw, n_ref=a.n_ref, precision=a.precision, dt_source=a.dt_source)
        ref = None
        if n1 > n0 > 0:
            # the wall coefficients' mean over steps n0 < n <= n1 of a plain
            # FP64 run from the free stream (from the library's running means)
            s = Solver(wl, stream=_stream().value)
            try:
                s.step(n0)
                sf0, cdr0 = s.surface(1)
                m0 = sf0[:, 3:6].copy()
                t0 = time.perf_counter()
                for k in range(n0, n1, 10000):
                    s.step(min(10000, n1 - k))
                    print(f"  reference: {min(k + 10000, n1)} steps {time.perf_counter() - t0:.1f} s", flush=True)
                sf1, cdr1 = s.surface(1)
                m1 = sf1[:, 3:6].copy()
            finally:
                s.close()
            ref = (n1 * m1 - n0 * m0) / (n1 - n0)
            ref_cd = (n1 * cdr1 - n0 * cdr0) / (n1 - n0)
            res["reference"] = dict(steps=[n0, n1], precision="f64", start="free stream")
        for start in a.starts.split(","):
            W0, info = (None, dict(seconds=0.0)) if start == "free" else warm_start(Ma, Kn, Tw, mlp, wl)
            s = Solver(wl, W0=W0, stream=_stream().value, precision=a.precision)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                conv, steps = s.step_until(a.target, a.max_steps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                surf, cd = s.surface(1)
                win = None
                if a.window > 0:
                    # means over a fixed window of steps after convergence,
                    # from the running means: (n1 M1 - n0 M0) / (n1 - n0)
                    n0c, m0c = int(steps), surf[:, 3:6].copy()
                    s.step(a.window)
                    s1, cd1 = s.surface(1)
                    n1c = n0c + a.window
                    win = ((n1c * s1[:, 3:6] - n0c * m0c) / a.window, (n1c * cd1 - n0c * cd) / a.window)
            finally:
                s.close()
            res[start] = dict(converged=conv, steps=int(steps), seconds=dt, start_seconds=info["seconds"],
                              cd_mean=cd)
            if win is not None:
                res[start]["window"] = dict(steps=a.window, cd=float(win[1]))
            if ref is not None:
                # relative L2 over the wall faces of the running means at convergence
                d = np.linalg.norm(surf[:, 3:6] - ref, axis=0) / np.linalg.norm(ref, axis=0)
                res[start].update(dCp=float(d[0]), dCF=float(d[1]), dCQ=float(d[2]))
                print(f"    wall means vs reference: dCp {d[0]:.3e} dCF {d[1]:.3e} dCQ {d[2]:.3e}", flush=True)
                if win is not None:
                    dw = np.linalg.norm(win[0] - ref, axis=0) / np.linalg.norm(ref, axis=0)
                    res[start]["window"].update(dCp=float(dw[0]), dCF=float(dw[1]), dCQ=float(dw[2]),
                                                dCd=float(abs(win[1] - ref_cd) / abs(ref_cd)))
                    print(f"    window of {a.window} steps vs reference: dCp {dw[0]:.3e} dCF {dw[1]:.3e} "
                          f"dCQ {dw[2]:.3e} dCd {res[start]['window']['dCd']:.3e}", flush=True)
            del W0
            print(f"  Ma {Ma:.2f} Kn {Kn:.4f} Tw {Tw:.3f} {start}: converged {conv} steps {steps} {dt:.1f} s "
                  f"(+{info['seconds']:.2f} s start) C_d {cd:.4f}", flush=True)
        out.append(res)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


def _march(s, target, max_steps, chunk, tag):
    """step_until in chunks with a progress line per chunk; returns
    (converged, steps, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv, n = False, 0
    while not conv and n < max_steps:
        conv, n = s.step_until(target, min(chunk, max_steps - n))
        print(f"    {tag}: step {n} r_avg {s.residual()[1]:.3e} {time.perf_counter() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    return conv, int(n), time.perf_counter() - t0


def cmd_batched(a):
    """Time to residual of several held-out cases: each case alone in plain
    FP64 from the free stream (leg "f64"), against all of them in one batched
    solve in the chosen precision from their warm starts (leg "batch-warm",
    the warm starts' time included) or from the free stream ("batch-free").
    A batch stops at the first step at which every case's r_avg is below the
    target; a single case at its own."""
    use_own_stream()
    cases = [tuple(c) for c in draws(a.n_test, 4)[: a.n_cases]]
    wls = [fine_case(Ma, Kn, Tw, n_ref=a.n_ref, seed=1) for (Ma, Kn, Tw) in cases]
    out = dict(cases=[dict(Ma=Ma, Kn=Kn, Tw=Tw) for (Ma, Kn, Tw) in cases], n_ref=a.n_ref, target=a.target)
    for leg in a.legs.split(","):
        if leg == "f64":
            per = []
            for (Ma, Kn, Tw), wl in zip(cases, wls):
                s = Solver(wl, stream=_stream().value)
                try:
                    conv, n, dt = _march(s, a.target, a.max_steps, a.chunk, f"f64 Ma {Ma:.2f}")
                finally:
                    s.close()
                per.append(dict(converged=conv, steps=n, seconds=dt))
            out[leg] = dict(precision="f64", start="free stream", cases=per,
                            seconds=sum(r["seconds"] for r in per), converged=all(r["converged"] for r in per))
        elif leg in ("batch-warm", "batch-free"):
            tws = 0.0
            batch = []
            mlp = MLP.load(a.weights) if leg == "batch-warm" else None
            for (Ma, Kn, Tw), wl in zip(cases, wls):
                w = dict(wl)
                if leg == "batch-warm":
                    W0, info = warm_start(Ma, Kn, Tw, mlp, wl)
                    w["W0"] = W0
                    tws += info["seconds"]
                batch.append(w)
            s = Solver.batch(batch, stream=_stream().value, precision=a.precision)
            try:
                conv, n, dt = _march(s, a.target, a.max_steps, a.chunk, leg)
                r_avg = [s.case_residual(k)[1] for k in range(len(batch))]
            finally:
                s.close()
            out[leg] = dict(precision=a.precision, start="warm start" if leg == "batch-warm" else "free stream",
                            converged=conv, steps=n, seconds=dt + tws, march_seconds=dt, warm_start_seconds=tws,
                            case_r_avg=r_avg)
        else:
            raise SystemExit(f"unknown leg {leg}")
        print(json.dumps({leg: out[leg]}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2607_09552_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    d = sub.add_parser("data")
    d.add_argument("--n-train", type=int, default=128)
    d.add_argument("--n-test", type=int, default=16)
    d.add_argument("--train-seed", type=int, default=3)
    d.add_argument("--n-ref", type=int, default=100)
    d.add_argument("--batch", type=int, default=48)
    d.add_argument("--transient", type=int, default=3000)
    d.add_argument("--average", type=int, default=2000)
    d.add_argument("--every", type=int, default=10)
    d.add_argument("--out", default="ws_data.npz")
    t = sub.add_parser("train")
    t.add_argument("--data", default="ws_data.npz", help="one or more data files, comma-separated")
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--batch", type=int, default=8192)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--log-every", type=int, default=500)
    t.add_argument("--out", default=WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--ma", type=float, default=0.0)
    e.add_argument("--kn", type=float, default=0.01)
    e.add_argument("--tw", type=float, default=0.2)
    e.add_argument("--n-test", type=int, default=16)
    e.add_argument("--n-cases", type=int, default=2)
    e.add_argument("--skip", type=int, default=0, help="start after the first SKIP held-out cases")
    e.add_argument("--n-ref", type=int, default=400)
    e.add_argument("--precision", default="mixed")
    e.add_argument("--starts", default="free,warm")
    e.add_argument("--target", type=float, default=1e-6)
    e.add_argument("--max-steps", type=int, default=200000)
    e.add_argument("--reference", default="",
                   help="N0,N1: compare the wall means with a plain FP64 run's mean over steps N0..N1")
    e.add_argument("--out", default="")
    e.add_argument("--window", type=int, default=0,
                   help="after convergence, compare the wall means over this many further steps")
    e.add_argument("--dt-source", choices=("initial", "freestream"), default="initial",
                   help="time steps of every run from its initial field (Eq. (33)) or from the freestream")
    b = sub.add_parser("batched", help="time to residual: cases alone in FP64 against one batched solve")
    b.add_argument("--weights", default=WEIGHTS)
    b.add_argument("--n-test", type=int, default=16)
    b.add_argument("--n-cases", type=int, default=4)
    b.add_argument("--n-ref", type=int, default=400)
    b.add_argument("--precision", default="mixed")
    b.add_argument("--legs", default="f64,batch-warm")
    b.add_argument("--target", type=float, default=1e-6)
    b.add_argument("--max-steps", type=int, default=200000)
    b.add_argument("--chunk", type=int, default=10000)
    b.add_argument("--out", default="")
    a = ap.parse_args(argv)
    sys.path.insert(0, ROOT)
    {"data": cmd_data, "train": cmd_train, "eval": cmd_eval, "batched": cmd_batched}[a.cmd](a)


if __name__ == "__main__":
    main()
