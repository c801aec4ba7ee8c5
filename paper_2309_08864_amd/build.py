"""Build libso2dr.so in-tree for gfx950 with hipcc (sources under csrc/).

Run as ``python -m paper_2309_08864_amd.build`` or through
``__graft_entry__.build()``.  Objects go to ``_build/`` beside this file; the
shared library lands next to this file, where ``_lib.py`` loads it.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libso2dr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(os.path.dirname(HERE), "include"), "-Wall", "-Wno-unused-function"]

# (source, extra compiler flags, object name): kernels.hip is compiled once
# per storage type (so2dr_dtype value in SO2DR_STORAGE)
SOURCES = [("kernels.hip", [f"-DSO2DR_STORAGE={d}"], f"kernels_{name}.o")
           for d, name in ((0, "f32"), (1, "f64"), (2, "bf16"), (3, "f16"))]
SOURCES += [(s, [], s + ".o") for s in ("aux_kernels.hip", "planner.cpp", "runtime.cpp",
                                         "adjoint.cpp", "model.cpp", "capi.cpp")]


def _deps_mtime(src: str) -> float:
    """Latest modification time of a source and of every header it can use
    (all headers of csrc/ and include/)."""
    inc = os.path.join(os.path.dirname(HERE), "include")
    files = [os.path.join(CSRC, src)]
    files += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    files += [os.path.join(inc, f) for f in os.listdir(inc)]
    return max(os.path.getmtime(f) for f in files)


def _compile(entry, incremental: bool = False) -> str:
    src, flags, objname = entry
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, objname)
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _deps_mtime(src):
        return obj
    cmd = [HIPCC] + COMMON + flags + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source and link libso2dr.so.  incremental=True keeps an
    object newer than its source and every header (a development shortcut;
    the default always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(jobs, 16)) as ex:
        objs = list(ex.map(lambda e: _compile(e, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
