"""UGKWP-LTS hot path on MI355X (gfx950): Python binding of libugkwp.so.

The binding only marshals arguments; every step of the method runs in the HIP
kernels of the library.  There is no CPU fallback: without the built library
(``python -m paper_2607_09552_amd.build``) or without a GPU, constructing a
Solver raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugkwp.so")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, ENUMERIC, ESTATE, EIO = 0, -1, -2, -3, -4, -5, -6, -7
BC_FARFIELD, BC_OUTFLOW, BC_WALL_DIFFUSE, BC_SYMMETRY = 1, 2, 3, 4

# Every entry point declared in include/ugkwp.h and include/ugkwp_mlp.h.
ABI_SYMBOLS = (
    "ugkwp_init", "ugkwp_init_batch", "ugkwp_case_range", "ugkwp_case_residual", "ugkwp_case_surface", "ugkwp_step", "ugkwp_step_until", "ugkwp_residual", "ugkwp_surface", "ugkwp_get_fields",
    "ugkwp_get_fields_device", "ugkwp_get_dt", "ugkwp_get_counts", "ugkwp_get_work", "ugkwp_get_particles",
    "ugkwp_set_particles", "ugkwp_set_fields", "ugkwp_set_step", "ugkwp_get_tally", "ugkwp_profile", "ugkwp_profile_read",
    "ugkwp_set_tuning", "ugkwp_get_tuning", "ugkwp_last_error", "ugkwp_free",
    "ugkwp_get_face_flux", "ugkwp_get_history", "ugkwp_set_history", "ugkwp_save", "ugkwp_load",
    "ugkwp_get_shakhov_fallbacks", "ugkwp_step_noalloc", "ugkwp_stream_copy",
    "ugkwp_mlp_layer", "ugkwp_mlp_gemm_acc", "ugkwp_mlp_act_backward", "ugkwp_mlp_adam", "ugkwp_mlp_to_bf16",
    "ugkwp_mlp_mse_grad", "ugkwp_ws_features", "ugkwp_ws_decode", "ugkwp_mlp_pack", "ugkwp_mlp_forward",
)


class UgkwpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ugkwp error {code}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_nodes", C.c_int64), ("nodes", C.c_void_p), ("n_cells", C.c_int64),
        ("cell_ptr", C.c_void_p), ("cell_nodes", C.c_void_p), ("n_bfaces", C.c_int64),
        ("bface_nodes", C.c_void_p), ("bface_type", C.c_void_p), ("bface_data", C.c_void_p),
    ]


class _Tuning(C.Structure):
    _fields_ = [("batch_steps", C.c_int32), ("use_graph", C.c_int32), ("transport_block", C.c_int32),
                ("shakhov_lanes", C.c_int32), ("max_crossings", C.c_int32), ("scatter_block", C.c_int32),
                ("tally_block", C.c_int32), ("flux_block", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [
        ("R", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double), ("T_ref", C.c_double),
        ("Pr", C.c_double), ("D", C.c_int32), ("cfl", C.c_double), ("n_ref", C.c_int32), ("lts", C.c_int32),
        ("seed", C.c_uint64), ("rho_inf", C.c_double), ("u_inf_x", C.c_double), ("u_inf_y", C.c_double),
        ("T_inf", C.c_double), ("L_ref", C.c_double), ("particle_capacity", C.c_int64), ("stream", C.c_void_p),
        ("precision", C.c_int32), ("wave_only", C.c_int32), ("dt_source", C.c_int32),
    ]


class WsCase(C.Structure):
    """ugkwp_ws_case: flow parameters and free stream of one warm-start case."""
    _fields_ = [("Ma", C.c_double), ("Kn", C.c_double), ("Tw", C.c_double), ("rho_inf", C.c_double),
                ("U_inf", C.c_double), ("T_inf", C.c_double), ("R", C.c_double), ("D", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libugkwp.so and declare its ABI.  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2607_09552_amd.build`")
    # torch bundles a HIP runtime under the same soname as the system one; the
    # first to load serves the whole process, and torch cannot use the system
    # runtime.  Loading torch first makes the library and torch share its.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, dp, i64p, i32p, u64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_uint64)
    L.ugkwp_init.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, C.POINTER(vp)]
    L.ugkwp_init_batch.argtypes = [C.c_int32, C.POINTER(_Mesh), C.POINTER(_Params), C.POINTER(dp), C.POINTER(vp)]
    L.ugkwp_case_range.argtypes = [vp, C.c_int32, i64p, i64p, i64p, i64p]
    L.ugkwp_case_residual.argtypes = [vp, C.c_int32, dp, dp]
    L.ugkwp_case_surface.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int64, i64p, dp]
    L.ugkwp_step.argtypes = [vp, C.c_int32]
    L.ugkwp_step_noalloc.argtypes = [vp, C.c_int32]
    L.ugkwp_step_until.argtypes = [vp, C.c_double, C.c_int32, i32p]
    L.ugkwp_residual.argtypes = [vp, dp, dp, i64p]
    L.ugkwp_surface.argtypes = [vp, C.c_int32, dp, C.c_int64, i64p, dp]
    L.ugkwp_get_fields.argtypes = [vp, dp]
    L.ugkwp_get_fields_device.argtypes = [vp, vp]
    L.ugkwp_get_dt.argtypes = [vp, dp]
    L.ugkwp_get_counts.argtypes = [vp, i32p, i64p, i64p, i64p, i64p, i64p]
    L.ugkwp_get_work.argtypes = [vp, i64p]
    L.ugkwp_get_particles.argtypes = [vp, C.c_int64, u64p, i32p, dp, dp, dp, dp, i64p]
    L.ugkwp_set_particles.argtypes = [vp, C.c_int64, u64p, i32p, dp, dp, dp, dp]
    L.ugkwp_get_tally.argtypes = [vp, dp, dp]
    L.ugkwp_set_fields.argtypes = [vp, dp]
    L.ugkwp_set_step.argtypes = [vp, C.c_int64]
    L.ugkwp_profile.argtypes = [vp, C.c_int32]
    L.ugkwp_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.ugkwp_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.ugkwp_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_char_p), dp, i64p, dp, i32p]
    L.ugkwp_get_face_flux.argtypes = [vp, dp, C.c_int64, i64p]
    L.ugkwp_get_history.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp]
    L.ugkwp_set_history.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp]
    L.ugkwp_save.argtypes = [vp, C.c_char_p]
    L.ugkwp_load.argtypes = [vp, C.c_char_p]
    L.ugkwp_get_shakhov_fallbacks.argtypes = [vp, i64p]
    L.ugkwp_stream_copy.argtypes = [vp, vp, C.c_int64, C.c_int32, C.c_int32, vp, dp]
    L.ugkwp_last_error.argtypes = [vp]
    L.ugkwp_last_error.restype = C.c_char_p
    L.ugkwp_free.argtypes = [vp]
    L.ugkwp_free.restype = None
    i64, i32, f32 = C.c_int64, C.c_int32, C.c_float
    L.ugkwp_mlp_layer.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp, vp, vp, vp, vp]
    L.ugkwp_mlp_gemm_acc.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp]
    L.ugkwp_mlp_act_backward.argtypes = [vp, vp, i64, i64, i32, vp, vp, vp, vp]
    L.ugkwp_mlp_adam.argtypes = [vp, vp, vp, vp, i64, i64, f32, f32, f32, f32, i64, vp, vp, vp]
    L.ugkwp_mlp_to_bf16.argtypes = [vp, i64, i64, vp, vp, vp]
    L.ugkwp_mlp_pack.argtypes = [vp, i64, i64, i32, vp, vp]
    L.ugkwp_mlp_forward.argtypes = [vp, i64, i32, C.POINTER(i32), C.POINTER(vp), C.POINTER(vp), vp, vp]
    L.ugkwp_mlp_mse_grad.argtypes = [vp, vp, i64, i64, i64, f32, vp, vp, vp]
    L.ugkwp_ws_features.argtypes = [vp, i32, i32, i32, i32, C.POINTER(WsCase), i64, vp, vp, vp, vp]
    L.ugkwp_ws_decode.argtypes = [vp, i64, vp, i64, C.POINTER(WsCase), vp, vp]
    _lib = L
    return L


def _ptr(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _vp(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def stream_copy(dst, src, reps=5, blocks=0):
    """Copies torch device tensor src into dst (same byte size) with the
    library's streaming kernel on torch's current stream; returns the mean
    milliseconds per copy (ugkwp_stream_copy)."""
    import torch
    L = load_library()
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_cuda and dst.is_cuda):
        raise ValueError("stream_copy: two device tensors of the same byte size")
    ms = C.c_double()
    rc = L.ugkwp_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nb, reps, blocks,
                             C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(ms))
    if rc != 0:
        raise UgkwpError(rc, "ugkwp_stream_copy failed")
    return ms.value


class Solver:
    """One UGKWP-LTS problem resident on the GPU.

    ``wl`` is a workload dict (see the ``workloads`` module).  ``stream`` is a
    raw hipStream_t handle (e.g. ``torch.cuda.current_stream().cuda_stream``)
    or None for the library's own stream.
    """

    def __init__(self, wl, W0=None, stream=None, particle_capacity=0, precision="f64", batch=None, tuned=True):
        L = load_library()
        self._keep = []
        # the workload(s), for host-side diagnostics: `cases` is the batch's
        # list of workloads (None for one case; `batch` is the constructor)
        self.wl, self.cases = wl, batch
        if batch is None:
            m, p, W = self._marshal(wl, W0, stream, particle_capacity, precision)
            self.dim, self.nc, self.ncase = int(wl["dim"]), int(wl["n_cells"]), 1
            h = C.c_void_p()
            rc = L.ugkwp_init(C.byref(m), C.byref(p), _ptr(W), C.byref(h))
        else:
            # a batch of independent cases (2D): `batch` is a list of workloads
            n = len(batch)
            ms, ps = (_Mesh * n)(), (_Params * n)()
            ws = (C.POINTER(C.c_double) * n)()
            for k, w in enumerate(batch):
                ms[k], ps[k], W = self._marshal(w, None, stream, particle_capacity, precision)
                ws[k] = _ptr(W)
            self.dim, self.nc, self.ncase = 2, int(sum(w["n_cells"] for w in batch)), n
            h = C.c_void_p()
            rc = L.ugkwp_init_batch(n, ms, ps, ws, C.byref(h))
        self.nw = self.dim + 2
        self.h = h
        if rc != OK:
            msg = L.ugkwp_last_error(h).decode() if h.value else ""
            self.close()
            raise UgkwpError(rc, msg)
        if tuned:
            from .autotune import load_tuning
            name = (wl or batch[0]).get("name") if (wl or batch) else None
            best = load_tuning(name) if name else None
            if best:
                self.set_tuning(**best)

    @classmethod
    def batch(cls, workloads, **kw):
        """One context holding independent cases; case k gives the results of
        Solver(workloads[k]) (same seeds)."""
        return cls(None, batch=list(workloads), **kw)

    def _marshal(self, wl, W0, stream, particle_capacity, precision):
        keep = self._keep

        def arr(a, dt):
            x = np.ascontiguousarray(a, dtype=dt)
            keep.append(x)
            return x

        dim = int(wl["dim"])
        m = _Mesh()
        m.dim = dim
        nodes = arr(wl["nodes"], np.float64).ravel()
        m.n_nodes = len(nodes) // dim
        m.nodes = _vp(nodes)
        m.n_cells = int(wl["n_cells"])
        if dim == 2:
            m.cell_ptr = _vp(arr(wl["cell_ptr"], np.int64))
            m.cell_nodes = _vp(arr(wl["cell_nodes"], np.int64))
        bt = arr(wl["bface_type"], np.int32)
        m.n_bfaces = len(bt)
        m.bface_nodes = _vp(arr(wl["bface_nodes"], np.int64).ravel())
        m.bface_type = _vp(bt)
        m.bface_data = _vp(arr(wl["bface_data"], np.float64).ravel())
        g, r = wl["gas"], wl["ref"]
        p = _Params(R=g["R"], omega=g["omega"], mu_ref=g["mu_ref"], T_ref=g["T_ref"], Pr=g["Pr"], D=g["D"],
                    cfl=wl["cfl"], n_ref=wl["n_ref"], lts=wl["lts"], seed=wl["seed"], rho_inf=r["rho_inf"],
                    u_inf_x=r["u_inf"][0], u_inf_y=r["u_inf"][1], T_inf=r["T_inf"], L_ref=r["L_ref"],
                    particle_capacity=particle_capacity, stream=stream,
                    precision={"f64": 0, "mixed": 1}[precision], wave_only=int(wl.get("wave_only", 0)),
                    dt_source=int(wl.get("dt_source", 0)))
        W = arr(wl["W0"] if W0 is None else W0, np.float64).ravel()
        return m, p, W

    def case_range(self, k):
        """(first cell, cells, first wall face, wall faces) of case k."""
        v = [C.c_int64() for _ in range(4)]
        self._check(load_library().ugkwp_case_range(self.h, k, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def case_residual(self, k):
        a, b = C.c_double(), C.c_double()
        self._check(load_library().ugkwp_case_residual(self.h, k, C.byref(a), C.byref(b)))
        return a.value, b.value

    def case_surface(self, k, mode=0):
        L = load_library()
        nw, cd = C.c_int64(), C.c_double()
        self._check(L.ugkwp_case_surface(self.h, k, mode, None, 0, C.byref(nw), C.byref(cd)))
        out = np.zeros((nw.value, 6))
        self._check(L.ugkwp_case_surface(self.h, k, mode, _ptr(out), nw.value, C.byref(nw), C.byref(cd)))
        return out, cd.value

    def _check(self, rc):
        if rc != OK:
            raise UgkwpError(rc, load_library().ugkwp_last_error(self.h).decode())

    def step(self, n=1):
        self._check(load_library().ugkwp_step(self.h, n))

    def step_noalloc(self, n=1):
        """ugkwp_step without any device allocation (scratch in the library's
        static array; no store growth, no graph replay)."""
        self._check(load_library().ugkwp_step_noalloc(self.h, n))

    def step_until(self, target, max_steps):
        """Steps until the first step n >= 100 with r_avg < target (r_inst in
        wave-only runs) or max_steps steps; returns (converged, steps done in
        total)."""
        conv = C.c_int32()
        self._check(load_library().ugkwp_step_until(self.h, target, max_steps, C.byref(conv)))
        return bool(conv.value), self.residual()[2]

    def fields(self):
        W = np.zeros((self.nc, self.nw))
        self._check(load_library().ugkwp_get_fields(self.h, _ptr(W)))
        return W

    def fields_device(self):
        """W as a float64 torch tensor on the GPU (stream-ordered copy)."""
        import torch
        out = torch.empty((self.nc, self.nw), dtype=torch.float64, device="cuda")
        self._check(load_library().ugkwp_get_fields_device(self.h, C.c_void_p(out.data_ptr())))
        return out

    def dt(self):
        d = np.zeros(self.nc)
        self._check(load_library().ugkwp_get_dt(self.h, _ptr(d)))
        return d

    def counts(self):
        cnt = np.zeros(self.nc, dtype=np.int32)
        v = [C.c_int64() for _ in range(5)]
        self._check(load_library().ugkwp_get_counts(self.h, _ptr(cnt, C.c_int32), *[C.byref(x) for x in v]))
        return cnt, dict(total=v[0].value, new=v[1].value, removed=v[2].value, exited=v[3].value, guard=v[4].value)

    def work(self):
        """Particles transported, summed over every step done."""
        n = C.c_int64()
        self._check(load_library().ugkwp_get_work(self.h, C.byref(n)))
        return n.value

    def particles(self):
        L = load_library()
        n = C.c_int64()
        L.ugkwp_get_particles(self.h, 0, None, None, None, None, None, None, C.byref(n))
        k = n.value
        pid = np.zeros(k, dtype=np.uint64)
        cell = np.zeros(k, dtype=np.int32)
        m = np.zeros(k)
        x = np.zeros((k, self.dim))
        u = np.zeros((k, 3))
        ei = np.zeros(k)
        self._check(L.ugkwp_get_particles(self.h, k, _ptr(pid, C.c_uint64), _ptr(cell, C.c_int32), _ptr(m), _ptr(x),
                                          _ptr(u), _ptr(ei), C.byref(n)))
        return dict(pid=pid, cell=cell, m=m, x=x, u=u, ei=ei)

    def set_particles(self, pid, cell, m, x, u, ei=None):
        pid = np.ascontiguousarray(pid, dtype=np.uint64)
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        m, x, u = (np.ascontiguousarray(a, dtype=np.float64) for a in (m, x, u))
        ei = None if ei is None else np.ascontiguousarray(ei, dtype=np.float64)
        self._check(load_library().ugkwp_set_particles(self.h, len(pid), _ptr(pid, C.c_uint64),
                                                       _ptr(cell, C.c_int32), _ptr(m), _ptr(x), _ptr(u), _ptr(ei)))

    def set_fields(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64)
        self._check(load_library().ugkwp_set_fields(self.h, _ptr(W)))

    def set_step(self, n):
        self._check(load_library().ugkwp_set_step(self.h, n))

    def residual(self):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        self._check(load_library().ugkwp_residual(self.h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def surface(self, mode=0):
        L = load_library()
        nw, cd = C.c_int64(), C.c_double()
        self._check(L.ugkwp_surface(self.h, mode, None, 0, C.byref(nw), C.byref(cd)))
        out = np.zeros((nw.value, 6))
        self._check(L.ugkwp_surface(self.h, mode, _ptr(out), nw.value, C.byref(nw), C.byref(cd)))
        return out, cd.value

    def stagnation(self, point, mode=2, case=0):
        """Wall pressure and heat-flux coefficients (C_p, C_Q) at a wall point
        (the stagnation point, Sec. V.A), linearly interpolated between the
        centres of the two wall faces nearest to it; mode as ugkwp_surface
        (2: the EMA with alpha = 2/1001, the paper's convergence monitor;
        interpolation and EMA commute).  A caller-side diagnostic: it
        post-processes the library's per-face output of ugkwp_surface on the
        host and is not part of the step."""
        out, _ = self.case_surface(case, mode) if self.ncase > 1 else self.surface(mode)
        d = np.hypot(out[:, 0] - point[0], out[:, 1] - point[1])
        a, b = np.argsort(d, kind="stable")[:2]
        wa = d[b] / (d[a] + d[b])
        return wa * out[a, 3] + (1.0 - wa) * out[b, 3], wa * out[a, 5] + (1.0 - wa) * out[b, 5]

    def face_flux(self):
        """Last committed step's F_j s_j per face [n_faces x (dim + 2)]."""
        L = load_library()
        nf = C.c_int64()
        self._check(L.ugkwp_get_face_flux(self.h, None, 0, C.byref(nf)))
        F = np.zeros((nf.value, self.nw))
        self._check(L.ugkwp_get_face_flux(self.h, _ptr(F), nf.value, C.byref(nf)))
        return F

    def n_wall(self):
        """Wall faces of the context (of every case of a batch)."""
        if self.ncase > 1:
            return sum(self.case_range(k)[3] for k in range(self.ncase))
        nw = C.c_int64()
        load_library().ugkwp_surface(self.h, 0, None, 0, C.byref(nw), None)
        return nw.value

    _HIST = ("rho_prev", "rho_sum", "rho_mean_prev", "wlast", "wsum", "wema", "scal")

    def history(self):
        """Averaging state: per-cell last density, density sum and running
        mean; per wall face last, summed and EMA (p, tau, q); per case the
        scalar results (r_inst, r_avg, C_d last, sum, EMA, unused)."""
        nwl = self.n_wall()
        h = dict(rho_prev=np.zeros(self.nc), rho_sum=np.zeros(self.nc), rho_mean_prev=np.zeros(self.nc),
                 wlast=np.zeros(3 * nwl), wsum=np.zeros(3 * nwl), wema=np.zeros(3 * nwl), scal=np.zeros(6 * self.ncase))
        self._check(load_library().ugkwp_get_history(self.h, *[_ptr(h[k]) for k in self._HIST]))
        return h

    def set_history(self, h):
        arrs = [None if h.get(k) is None else np.ascontiguousarray(h[k], dtype=np.float64) for k in self._HIST]
        self._check(load_library().ugkwp_set_history(self.h, *[_ptr(a) for a in arrs]))

    def save(self, path):
        self._check(load_library().ugkwp_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._check(load_library().ugkwp_load(self.h, os.fsencode(path)))

    def shakhov_fallbacks(self):
        n = C.c_int64()
        self._check(load_library().ugkwp_get_shakhov_fallbacks(self.h, C.byref(n)))
        return n.value

    def tally(self):
        Sm = np.zeros((self.nc, self.nw))
        Sp = np.zeros((self.nc, self.nw))
        self._check(load_library().ugkwp_get_tally(self.h, _ptr(Sm), _ptr(Sp)))
        return Sm, Sp

    def tuning(self):
        t = _Tuning()
        self._check(load_library().ugkwp_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = _Tuning(**cur)
        self._check(load_library().ugkwp_set_tuning(self.h, C.byref(t)))

    def profile(self, enable=True, transport_only=False):
        mode = 0 if not enable else (2 if transport_only else 1)
        self._check(load_library().ugkwp_profile(self.h, mode))

    def profile_read(self):
        L = load_library()
        cap = 32
        names = (C.c_char_p * cap)()
        ms = np.zeros(cap)
        nl = np.zeros(cap, dtype=np.int64)
        by = np.zeros(cap)
        n = C.c_int32()
        self._check(L.ugkwp_profile_read(self.h, cap, names, _ptr(ms), _ptr(nl, C.c_int64), _ptr(by), C.byref(n)))
        return {names[k].decode(): dict(ms=ms[k], launches=int(nl[k]), bytes=by[k]) for k in range(n.value)}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load_library().ugkwp_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
