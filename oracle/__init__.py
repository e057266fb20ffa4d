"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
import this module.  It shares no code with the HIP product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libugkwp_oracle.so")
SRC = os.path.join(HERE, "ugkwp_oracle.c")

OK, EINVAL, ENOMEM, EOVERFLOW, ENUMERIC = 0, -1, -2, -4, -5


def build(quiet: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle with gcc: serial, FP64, no contraction, no fast-math.

    sanitize=True adds AddressSanitizer and UndefinedBehaviorSanitizer
    (-fsanitize=address,undefined, frame pointers kept); such a build must be
    loaded into a process started with the sanitizer runtimes preloaded
    (LD_PRELOAD of libasan and libubsan, see sanitizer_env()).  `out` names
    the library to write (default: the one lib() loads)."""
    target = out or LIB
    flags = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-fPIC", "-shared"]
    if sanitize:
        flags += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = ["gcc", *flags, "-o", target + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(target + ".tmp", target)
    return target


def sanitizer_env() -> dict:
    """Environment for a child process that loads a sanitize=True build:
    LD_PRELOAD of gcc's ASan and UBSan runtimes, leak checking off (the
    Python interpreter itself is not leak-clean), and the build's path in
    UGKWP_ORACLE_LIB so that lib() loads it."""
    def runtime(name):
        r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
        return r.stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join([runtime("libasan.so"), runtime("libubsan.so")])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


class _Mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n_nodes", C.c_int64),
        ("nodes", C.POINTER(C.c_double)),
        ("n_cells", C.c_int64),
        ("cell_ptr", C.POINTER(C.c_int64)),
        ("cell_nodes", C.POINTER(C.c_int64)),
        ("n_bfaces", C.c_int64),
        ("bface_nodes", C.POINTER(C.c_int64)),
        ("bface_type", C.POINTER(C.c_int32)),
        ("bface_data", C.POINTER(C.c_double)),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("R", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double), ("T_ref", C.c_double),
        ("Pr", C.c_double), ("D", C.c_int32), ("cfl", C.c_double), ("n_ref", C.c_int32),
        ("lts", C.c_int32), ("seed", C.c_uint64), ("rho_inf", C.c_double), ("u_inf_x", C.c_double),
        ("u_inf_y", C.c_double), ("T_inf", C.c_double), ("L_ref", C.c_double), ("wave_only", C.c_int32),
        ("dt_source", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("UGKWP_ORACLE_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        dp, ip64, ip32, up64 = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_uint64)
        L.ref_init.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, C.POINTER(C.c_void_p)]
        L.ref_step.argtypes = [C.c_void_p, C.c_int32]
        L.ref_get_fields.argtypes = [C.c_void_p, dp]
        L.ref_set_fields.argtypes = [C.c_void_p, dp]
        L.ref_get_dt.argtypes = [C.c_void_p, dp]
        L.ref_get_counts.argtypes = [C.c_void_p, ip32, ip64, ip64, ip64, ip64]
        L.ref_get_particles.argtypes = [C.c_void_p, C.c_int64, up64, ip32, dp, dp, dp, dp, ip64]
        L.ref_set_particles.argtypes = [C.c_void_p, C.c_int64, up64, ip32, dp, dp, dp, dp]
        L.ref_residual.argtypes = [C.c_void_p, dp, dp, ip64]
        L.ref_surface.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64, ip64, dp]
        L.ref_get_tally.argtypes = [C.c_void_p, dp, dp]
        L.ref_get_face_flux.argtypes = [C.c_void_p, dp]
        L.ref_n_faces.argtypes = [C.c_void_p]
        L.ref_n_faces.restype = C.c_int64
        L.ref_n_guard.argtypes = [C.c_void_p]
        L.ref_n_guard.restype = C.c_int64
        L.ref_set_step.argtypes = [C.c_void_p, C.c_int64]
        L.ref_set_step.restype = None
        L.ref_last_error.argtypes = [C.c_void_p]
        L.ref_last_error.restype = C.c_char_p
        L.ref_free.argtypes = [C.c_void_p]
        L.ref_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.ref_uniform.argtypes = [C.c_uint32, C.c_uint32]
        L.ref_uniform.restype = C.c_double
        L.ref_time_coeffs.argtypes = [C.c_double, C.c_double, dp]
        L.ref_moments_n.argtypes = [C.c_double, C.c_double, C.c_int, dp]
        L.ref_microslope.argtypes = [dp, dp, C.c_int, C.c_double, dp]
        L.ref_flux_interior.argtypes = [dp, dp, dp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_int, C.c_double, C.c_int, dp, dp]
        L.ref_flux_wall.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.ref_track_one.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, C.c_int32, dp, dp, dp, C.c_double,
                                    ip32, ip32]
        L.ref_exact_sum.argtypes = [dp, C.c_int64]
        L.ref_exact_sum.restype = C.c_double
        L.ref_reconstruct.argtypes = [dp, C.c_double, dp, C.c_double, dp, C.c_double, C.c_int, dp, dp]
        L.ref_reconstruct.restype = None
        L.ref_face_values.argtypes = [C.c_void_p, C.c_int64, dp, dp, dp, dp, dp]
        L.ref_face_geom.argtypes = [C.c_void_p, C.c_int64, dp]
        L.ref_vacuum_guard.argtypes = [C.c_void_p, dp, C.c_double, dp]
        L.ref_sample_deviation.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, dp, C.c_double, dp, dp]
        L.ref_n_capped.argtypes = [C.c_void_p]
        L.ref_n_capped.restype = C.c_int64
        L.ref_get_history.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp, dp]
        L.ref_set_history.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# stage-level helpers
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().ref_philox4x32_10(c, k, o)
    return list(o)


def uniform(a, b):
    return lib().ref_uniform(a & 0xFFFFFFFF, b & 0xFFFFFFFF)


def time_coeffs(dt, tau):
    out = np.zeros(8)
    lib().ref_time_coeffs(dt, tau, _p(out))
    return out


def moments_n(U, lam, sign):
    out = np.zeros(7)
    lib().ref_moments_n(U, lam, sign, _p(out))
    return out


def microslope(W, dW, K=1, Pr=1.0):
    W, dW, a = _f64(W), _f64(dW), np.zeros(4)
    lib().ref_microslope(_p(W), _p(dW), K, Pr, _p(a))
    return a


def flux_interior(WL, WR, dW0, WhL, WhR, dWhL, dWhR, dtL, tauL, dtR, tauR, K=1, Pr=1.0, wave_only=0):
    WL, WR, dW0 = _f64(WL), _f64(WR), _f64(dW0)
    WhL = None if WhL is None else _f64(WhL)
    WhR = None if WhR is None else _f64(WhR)
    dWhL, dWhR = _f64(dWhL), _f64(dWhR)
    Feq, Ffr = np.zeros(4), np.zeros(4)
    lib().ref_flux_interior(_p(WL), _p(WR), _p(dW0), _p(WhL), _p(WhR), _p(dWhL), _p(dWhR), dtL, tauL, dtR,
                            tauR, K, Pr, wave_only, _p(Feq), _p(Ffr))
    return Feq, Ffr


def exact_sum(x):
    x = _f64(x)
    return lib().ref_exact_sum(_p(x), len(x))


def reconstruct(Wfar, xfar, Wself, xself, Wother, xother, K=1):
    Wfar = None if Wfar is None else _f64(Wfar)
    Wself, Wother = _f64(Wself), _f64(Wother)
    out, slope = np.zeros(4), np.zeros(4)
    lib().ref_reconstruct(_p(Wfar), xfar, _p(Wself), xself, _p(Wother), xother, K, _p(out), _p(slope))
    return out, slope


def flux_wall(W, Wh, dt, tau, Tw, R=1.0, K=1, wave_only=0):
    W = _f64(W)
    Wh = None if Wh is None else _f64(Wh)
    F = np.zeros(4)
    lib().ref_flux_wall(_p(W), _p(Wh), dt, tau, Tw, R, K, wave_only, _p(F))
    return F


# ---------------------------------------------------------------------------
# whole-step solver
# ---------------------------------------------------------------------------

class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """Serial FP64 UGKWP-LTS on the CPU for one workload dict."""

    def __init__(self, wl, W0=None):
        L = lib()
        self.wl = wl
        self.dim = int(wl["dim"])
        self.nw = self.dim + 2
        self._keep = []
        m = _Mesh()
        m.dim = self.dim
        nodes = _f64(wl["nodes"]).ravel()
        m.n_nodes = len(nodes) // self.dim
        m.nodes = _p(nodes)
        m.n_cells = int(wl["n_cells"])
        if self.dim == 2:
            cp = np.ascontiguousarray(wl["cell_ptr"], dtype=np.int64)
            cn = np.ascontiguousarray(wl["cell_nodes"], dtype=np.int64)
            m.cell_ptr, m.cell_nodes = _p(cp, C.c_int64), _p(cn, C.c_int64)
            self._keep += [cp, cn]
        bn = np.ascontiguousarray(wl["bface_nodes"], dtype=np.int64).ravel()
        bt = np.ascontiguousarray(wl["bface_type"], dtype=np.int32)
        bd = _f64(wl["bface_data"]).ravel()
        m.n_bfaces = len(bt)
        m.bface_nodes, m.bface_type, m.bface_data = _p(bn, C.c_int64), _p(bt, C.c_int32), _p(bd)
        self._keep += [nodes, bn, bt, bd]
        g = wl["gas"]
        r = wl["ref"]
        p = _Params(R=g["R"], omega=g["omega"], mu_ref=g["mu_ref"], T_ref=g["T_ref"], Pr=g["Pr"], D=g["D"],
                    cfl=wl["cfl"], n_ref=wl["n_ref"], lts=wl["lts"], seed=wl["seed"], rho_inf=r["rho_inf"],
                    u_inf_x=r["u_inf"][0], u_inf_y=r["u_inf"][1], T_inf=r["T_inf"], L_ref=r["L_ref"],
                    wave_only=int(wl.get("wave_only", 0)), dt_source=int(wl.get("dt_source", 0)))
        W = _f64(wl["W0"] if W0 is None else W0).ravel()
        h = C.c_void_p()
        rc = L.ref_init(C.byref(m), C.byref(p), _p(W), C.byref(h))
        self.h = h
        self.nc = int(wl["n_cells"])
        if rc != OK:
            msg = L.ref_last_error(h).decode() if h.value else ""
            self.close()
            raise OracleError(rc, msg)
        self.nf = int(L.ref_n_faces(h))

    def _check(self, rc):
        if rc != OK:
            raise OracleError(rc, lib().ref_last_error(self.h).decode())

    def step(self, n=1):
        self._check(lib().ref_step(self.h, n))

    def fields(self):
        W = np.zeros((self.nc, self.nw))
        lib().ref_get_fields(self.h, _p(W))
        return W

    def set_fields(self, W):
        W = _f64(W)
        lib().ref_set_fields(self.h, _p(W))

    def dt(self):
        d = np.zeros(self.nc)
        lib().ref_get_dt(self.h, _p(d))
        return d

    def counts(self):
        cnt = np.zeros(self.nc, dtype=np.int32)
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        lib().ref_get_counts(self.h, _p(cnt, C.c_int32), C.byref(a), C.byref(b), C.byref(c), C.byref(d))
        return cnt, dict(total=a.value, new=b.value, removed=c.value, exited=d.value,
                         guard=int(lib().ref_n_guard(self.h)))

    def particles(self):
        n = C.c_int64()
        lib().ref_get_particles(self.h, 0, None, None, None, None, None, None, C.byref(n))
        k = n.value
        pid = np.zeros(k, dtype=np.uint64)
        cell = np.zeros(k, dtype=np.int32)
        m = np.zeros(k)
        x = np.zeros((k, self.dim))
        u = np.zeros((k, 3))
        ei = np.zeros(k)
        self._check(lib().ref_get_particles(self.h, k, _p(pid, C.c_uint64), _p(cell, C.c_int32), _p(m), _p(x),
                                            _p(u), _p(ei), C.byref(n)))
        return dict(pid=pid, cell=cell, m=m, x=x, u=u, ei=ei)

    def set_particles(self, pid, cell, m, x, u, ei=None):
        pid = np.ascontiguousarray(pid, dtype=np.uint64)
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        m, x, u = _f64(m), _f64(x), _f64(u)
        ei = None if ei is None else _f64(ei)
        self._check(lib().ref_set_particles(self.h, len(pid), _p(pid, C.c_uint64), _p(cell, C.c_int32), _p(m),
                                            _p(x), _p(u), None if ei is None else _p(ei)))

    def set_step(self, n):
        lib().ref_set_step(self.h, n)

    def residual(self):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        lib().ref_residual(self.h, C.byref(a), C.byref(b), C.byref(n))
        return a.value, b.value, n.value

    def surface(self, mode=0):
        nw = C.c_int64()
        cd = C.c_double()
        lib().ref_surface(self.h, mode, None, 0, C.byref(nw), C.byref(cd))
        out = np.zeros((nw.value, 6))
        self._check(lib().ref_surface(self.h, mode, _p(out), nw.value, C.byref(nw), C.byref(cd)))
        return out, cd.value

    def tally(self):
        Sm = np.zeros((self.nc, self.nw))
        Sp = np.zeros((self.nc, self.nw))
        lib().ref_get_tally(self.h, _p(Sm), _p(Sp))
        return Sm, Sp

    def face_values(self, fi):
        """(W_L, W_R, slope_L, slope_R, dW0) of interior face fi, face frame."""
        out = [np.zeros(4) for _ in range(5)]
        self._check(lib().ref_face_values(self.h, fi, *[_p(a) for a in out]))
        return out

    def face_geom(self, fi):
        """dict(L, R, LL, RR, mid=(x, y), n=(nx, ny)) of face fi."""
        g = np.zeros(8)
        self._check(lib().ref_face_geom(self.h, fi, _p(g)))
        return dict(L=int(g[0]), R=int(g[1]), LL=int(g[2]), RR=int(g[3]), mid=g[4:6].copy(), n=g[6:8].copy())

    def vacuum_guard(self, Sp, vol, Wn):
        Sp, Wn = _f64(Sp), _f64(Wn).copy()
        fired = lib().ref_vacuum_guard(self.h, _p(Sp), vol, _p(Wn))
        return bool(fired), Wn

    def sample_deviation(self, pid, step, Uh, Th, shak=None):
        Uh = _f64(Uh)
        shak = None if shak is None else _f64(shak)
        z = np.zeros(3)
        capped = lib().ref_sample_deviation(self.h, pid, step, _p(Uh), Th, _p(shak), _p(z))
        return z, bool(capped)

    def n_capped(self):
        return int(lib().ref_n_capped(self.h))

    def n_wall(self):
        nw = C.c_int64()
        lib().ref_surface(self.h, 0, None, 0, C.byref(nw), None)
        return nw.value

    def history(self):
        nwl = self.n_wall()
        h = dict(rho_prev=np.zeros(self.nc), rho_sum=np.zeros(self.nc), rho_mean_prev=np.zeros(self.nc),
                 wlast=np.zeros(3 * nwl), wsum=np.zeros(3 * nwl), wema=np.zeros(3 * nwl), cd=np.zeros(3))
        lib().ref_get_history(self.h, *[_p(h[k]) for k in ("rho_prev", "rho_sum", "rho_mean_prev", "wlast", "wsum",
                                                               "wema", "cd")])
        return h

    def set_history(self, h):
        keys = ("rho_prev", "rho_sum", "rho_mean_prev", "wlast", "wsum", "wema", "cd")
        arrs = [None if h.get(k) is None else _f64(h[k]) for k in keys]
        lib().ref_set_history(self.h, *[_p(a) for a in arrs])

    def face_flux(self):
        F = np.zeros((self.nf, self.nw))
        lib().ref_get_face_flux(self.h, _p(F))
        return F

    def track_one(self, pid, step, cell, x, u, m, t):
        x2 = np.zeros(2)
        x2[: len(x)] = x
        u3 = _f64(u).copy()
        mm = C.c_double(m)
        co, nx = C.c_int32(), C.c_int32()
        rc = lib().ref_track_one(self.h, pid, step, cell, _p(x2), _p(u3), C.byref(mm), t, C.byref(co), C.byref(nx))
        return dict(rc=rc, cell=co.value, x=x2[: self.dim].copy(), u=u3, m=mm.value, ncross=nx.value)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ref_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
