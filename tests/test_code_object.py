"""The gfx950 code the library was built into (its own build, read with the
ROCm LLVM tools; no GPU): no packed FP32 arithmetic, which the build turns
off because some of its forms have given wrong results on this hardware,
and matrix-core (MFMA) instructions in the warm-start network's kernels."""
import os
import re
import shutil
import subprocess

import pytest

LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _disassembly(lib, tmp):
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")]
    if not all(os.path.exists(t) for t in tools):
        pytest.skip("ROCm LLVM tools not available")
    objcopy, bundler, objdump = tools
    fat = os.path.join(tmp, "fatbin.bin")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", lib, os.path.join(tmp, "copy.so")],
                   check=True, capture_output=True)
    data = open(fat, "rb").read()
    offs = [m.start() for m in re.finditer(re.escape(MAGIC), data)] + [len(data)]
    out = []
    for k in range(len(offs) - 1):  # one bundle per translation unit
        b, co = os.path.join(tmp, f"b{k}.bin"), os.path.join(tmp, f"co{k}.o")
        open(b, "wb").write(data[offs[k]:offs[k + 1]])
        subprocess.run([bundler, "--unbundle", "--type=o", f"--input={b}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True,
                       capture_output=True)
        out.append(subprocess.run([objdump, "-d", "--mcpu=gfx950", co], check=True, capture_output=True,
                                  text=True).stdout)
    return out


def test_code_object_has_no_packed_fp32_and_uses_mfma(tmp_path):
    import paper_2607_09552_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    dis = _disassembly(pkg.LIB_PATH, str(tmp_path))
    assert len(dis) == 3  # kernels.hip, api.hip, mlp.hip
    text = "\n".join(dis)
    assert "k_transport" in text and "k_scatter" in text and "k_layer" in text
    assert not re.findall(r"\bv_pk_(?:fma|add|mul)_f32\b", text)
    assert len(re.findall(r"\bv_mfma_\w+", text)) > 0
