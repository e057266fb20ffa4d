"""The C ABI library loads and exports every entry point include/*.h
declares, its structs, codes and argument checks agree with the binding
(no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ugkwp_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_step_api():
    names = declared_functions()
    for required in ("ugkwp_init", "ugkwp_step", "ugkwp_residual", "ugkwp_surface"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2607_09552_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pkg.ABI_SYMBOLS) == names


def test_solver_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2607_09552_amd as pkg
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pkg.load_library(str(tmp_path / "nope.so"))


def test_library_exports_no_other_c_symbols():
    """Only the declared entry points are exported with C linkage."""
    import shutil
    import subprocess
    import paper_2607_09552_amd as pkg
    if shutil.which("nm") is None or not os.path.exists(pkg.LIB_PATH):
        pytest.skip("nm or the library is not available")
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[1] in "TW"}
    c_syms = {x for x in syms if not x.startswith("_")}
    assert c_syms == set(declared_functions()), sorted(c_syms ^ set(declared_functions()))


def _struct_fields(header, name):
    """(field, ctypes type) pairs, in order, of `typedef struct { ... } name;`
    in a header (pointers as c_void_p)."""
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", header)).read(), flags=re.S)
    end = re.search(r"\}\s*" + name + r"\s*;", src).start()
    body = src[src.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "uint64_t": ctypes.c_uint64,
             "double": ctypes.c_double}
    fields = []
    for decl in body.split(";"):
        m = re.match(r"\s*(?:const\s+)?(\w+)\s+(.*\S)", decl, flags=re.S)
        if not m:
            continue
        for d in m.group(2).split(","):
            d = d.strip()
            fields.append((d.lstrip("*").strip(), ctypes.c_void_p if d.startswith("*") else ctype[m.group(1)]))
    return fields


@pytest.mark.parametrize("header, struct, cls", [("ugkwp.h", "ugkwp_tuning", "_Tuning"),
                                                 ("ugkwp.h", "ugkwp_params", "_Params"),
                                                 ("ugkwp.h", "ugkwp_mesh", "_Mesh"),
                                                 ("ugkwp_mlp.h", "ugkwp_ws_case", "WsCase")])
def test_structs_match_the_binding(header, struct, cls):
    """The binding's ctypes layouts follow the headers field for field and
    type for type, so a field added or retyped on one side only is caught."""
    import paper_2607_09552_amd as pkg
    assert _struct_fields(header, struct) == list(getattr(pkg, cls)._fields_)


def test_recorded_tuning_uses_known_fields():
    """Every setting in the recorded tuning table is a field of ugkwp_tuning."""
    import json
    import paper_2607_09552_amd as pkg
    from paper_2607_09552_amd import autotune
    known = {n for n, _ in pkg._Tuning._fields_}
    data = json.load(open(autotune.TUNING_FILE))
    for name, rec in data.items():
        assert set(rec["best"]) <= known, (name, set(rec["best"]) - known)
    assert set(autotune.SPACE) <= known


def _enum_values(path, prefix):
    """NAME -> value of the `PREFIX_NAME = value` enumerators in a header."""
    src = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b" + prefix + r"_(\w+)\s*=\s*(-?\d+)", src)}


def test_codes_match_the_header():
    """The status and boundary-type codes the binding, the workload builders
    and the oracle use are the values include/ugkwp.h gives them: a workload
    built once feeds both the library and the oracle."""
    import paper_2607_09552_amd as pkg
    import workloads
    lib = _enum_values(os.path.join(ROOT, "include", "ugkwp.h"), "UGKWP")
    ref = _enum_values(os.path.join(ROOT, "oracle", "ugkwp_oracle.h"), "REF")
    status = ("OK", "EINVAL", "ENOMEM", "EDEVICE", "EOVERFLOW", "ENUMERIC", "ESTATE", "EIO")
    assert {k: lib[k] for k in status} == {k: getattr(pkg, k) for k in status}
    assert len(set(lib[k] for k in status)) == len(status)
    for k in ("OK", "EINVAL", "ENOMEM", "EOVERFLOW", "ENUMERIC"):
        assert ref[k] == lib[k], k
    bc = {k: v for k, v in lib.items() if k.startswith("BC_")}
    assert set(bc) == {"BC_FARFIELD", "BC_OUTFLOW", "BC_WALL_DIFFUSE", "BC_SYMMETRY", "BC_WALL_MAXWELL"}
    for k, v in bc.items():
        assert getattr(workloads, k) == v, k
        if hasattr(pkg, k):
            assert getattr(pkg, k) == v, k
    assert ref["BC_WALL"] == bc["BC_WALL_DIFFUSE"]
    for k in ("BC_FARFIELD", "BC_OUTFLOW", "BC_SYMMETRY", "BC_WALL_MAXWELL"):
        assert ref[k] == bc[k], k


def _ctx_entry_points():
    """Entry points of include/ugkwp.h whose first argument is the context."""
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "ugkwp.h")).read(), flags=re.S)
    return re.findall(r"\bint\s+(ugkwp_\w+)\s*\(\s*(?:const\s+)?ugkwp_ctx\s*\*", src)


def test_entry_points_reject_a_null_context():
    """Every call on a context returns EINVAL for a null one, before any
    device call (so this runs without a GPU); the binding declares the
    argument types of each."""
    import paper_2607_09552_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    L = pkg.load_library()
    names = _ctx_entry_points()
    assert len(names) >= 25 and "ugkwp_step_noalloc" in names
    ints = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64)
    for n in names:
        f = getattr(L, n)
        assert f.argtypes is not None, n
        args = [0.0 if t is ctypes.c_double else 0 if t in ints else None for t in f.argtypes]
        assert f(*args) == pkg.EINVAL, n
    assert L.ugkwp_last_error(None) == b"no context"
    L.ugkwp_free(None)
    assert L.ugkwp_stream_copy(None, None, 0, 1, 0, None, None) == pkg.EINVAL


def test_init_rejects_bad_arguments_before_any_device_call():
    """ugkwp_init and ugkwp_init_batch check their arguments on the host:
    the error comes back with a context that says why and frees without a
    device."""
    import paper_2607_09552_amd as pkg
    import workloads
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    L = pkg.load_library()
    assert L.ugkwp_init(None, None, None, None) == pkg.EINVAL

    def fails(rc, h, text):
        assert rc == pkg.EINVAL and h.value
        msg = L.ugkwp_last_error(h).decode()
        L.ugkwp_free(h)
        assert text in msg, msg

    h = ctypes.c_void_p()
    fails(L.ugkwp_init(None, None, None, ctypes.byref(h)), h, "null argument")
    s = pkg.Solver.__new__(pkg.Solver)
    s._keep = []
    m, p, W = s._marshal(workloads.shock1d(n_half=8), None, None, 0, "f64")
    Wp = W.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for field, bad in (("cfl", 0.0), ("n_ref", 0), ("R", -1.0), ("dt_source", 2)):
        good = getattr(p, field)
        setattr(p, field, bad)
        fails(L.ugkwp_init(ctypes.byref(m), ctypes.byref(p), Wp, ctypes.byref(h)), h, "invalid parameters")
        setattr(p, field, good)
    m.dim = 3
    fails(L.ugkwp_init(ctypes.byref(m), ctypes.byref(p), Wp, ctypes.byref(h)), h, "dim must be 1 or 2")

    box = workloads.box2d(np.linspace(0.0, 1.0, 5), np.linspace(0.0, 1.0, 4))
    cases = [workloads.uniform2d(box), workloads.uniform2d(box, cfl=0.5)]
    ms, ps = (pkg._Mesh * 2)(), (pkg._Params * 2)()
    ws = (ctypes.POINTER(ctypes.c_double) * 2)()
    for k, w in enumerate(cases):
        ms[k], ps[k], Wk = s._marshal(w, None, None, 0, "f64")
        ws[k] = Wk.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fails(L.ugkwp_init_batch(0, ms, ps, ws, ctypes.byref(h)), h, "no case")
    fails(L.ugkwp_init_batch(2, ms, ps, ws, ctypes.byref(h)), h, "must equal case 0's")


def _prototypes():
    """(return type, name, [ctypes type per argument]) of every function the
    headers declare; pointers as c_void_p."""
    scalar = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "uint64_t": ctypes.c_uint64,
              "double": ctypes.c_double, "float": ctypes.c_float}
    out = []
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for ret, name, args in re.findall(r"\b(int|void|const\s+char\s*\*)\s*(ugkwp_\w+)\s*\(([^)]*)\)\s*;", src):
            types = []
            for a in (x.strip() for x in args.split(",") if x.strip()):
                if "*" in a:
                    types.append(ctypes.c_void_p)
                else:
                    types.append(scalar[re.sub(r"\bconst\b", "", a).split()[0]])
            out.append((ret, name, types))
    return out


def test_every_entry_point_rejects_null_arguments():
    """With null pointers and zero sizes every entry point of both headers
    returns EINVAL (-1) from its host-side checks, before any device call."""
    import paper_2607_09552_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    pkg.load_library()  # torch's HIP runtime first, as the binding loads it
    lib = ctypes.CDLL(pkg.LIB_PATH)  # own handle: argument types set here stay here
    protos = _prototypes()
    assert {n for _, n, _ in protos} == set(declared_functions())
    checked = 0
    for ret, name, types in protos:
        if ret != "int":
            continue
        f = getattr(lib, name)
        f.argtypes, f.restype = types, ctypes.c_int
        args = [None if t is ctypes.c_void_p else t(0) for t in types]
        assert f(*args) == pkg.EINVAL, name
        checked += 1
    assert checked >= 40


def test_tuning_values_within_the_library_ranges():
    """Every recorded best setting and every value the tuner sweeps is one
    ugkwp_set_tuning accepts (block sizes 64, 128 or 256, the re-sort also
    512; Shakhov lanes 1 to 16 in powers of two; 1 to 1024 steps per batch;
    graph on or off; 1 to 10000 crossings), so a sweep never stops on an
    EINVAL and a recorded table always loads."""
    import json
    from paper_2607_09552_amd import autotune
    ok = {"transport_block": {64, 128, 256}, "tally_block": {64, 128, 256}, "flux_block": {64, 128, 256},
          "scatter_block": {64, 128, 256, 512}, "shakhov_lanes": {1, 2, 4, 8, 16}, "use_graph": {0, 1},
          "batch_steps": set(range(1, 1025)), "max_crossings": set(range(1, 10001))}
    for name, values in autotune.SPACE.items():
        assert set(values) <= ok[name], name
    for case, rec in json.load(open(autotune.TUNING_FILE)).items():
        for name, v in rec["best"].items():
            assert v in ok[name], (case, name, v)
        for key in rec.get("seconds_per_update", {}):
            for name, v in json.loads(key).items():
                assert v in ok[name], (case, name, v)
