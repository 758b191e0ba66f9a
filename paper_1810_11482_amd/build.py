"""Build libhx.so: the HIP kernels and the C++ runtime behind include/hx.h.

Every HIP translation unit is compiled for gfx950 with hipcc; the host-only
C++ files too (they use the HIP runtime API).  The library links the HIP
runtime and runtime compiler that the installed PyTorch ships
(torch/lib/libamdhip64.so, libhiprtc.so), so a process that uses torch for
device memory and streams and this library for the kernels has exactly one HIP
runtime loaded.

Usage: python paper_1810_11482_amd/build.py  (run as a file: importing the package
loads the library this script builds)
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "hx")
LIB = os.path.join(HERE, "libhx.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]
# Device code: gfx950 only; packed FP32 instructions disabled.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("torch is required: libhx links the HIP runtime torch ships")
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    for lib in ("libamdhip64.so", "libhiprtc.so"):
        if not os.path.exists(os.path.join(d, lib)):
            raise RuntimeError(f"no {lib} in {d}")
    return d


def _up_to_date(src: str, obj: str) -> bool:
    """The object is newer than its source and every header it may include."""
    if not os.path.exists(obj):
        return False
    deps = [src] + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(CSRC, "*.hpp")) \
        + glob.glob(os.path.join(INCLUDE, "*.h"))
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if incremental and _up_to_date(src, obj):
        return obj
    if src.endswith(".hip"):
        cmd = [HIPCC, *COMMON, *DEVICE, "-c", src, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-x", "c++", "-c", src,
               "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, only those whose object is
    older than the source or a header) and link libhx.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    # the slowest translation units first, so they do not start last
    srcs.sort(key=lambda f: -os.path.getsize(f))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
    tlib = _torch_lib_dir()
    tmp = LIB + f".tmp{os.getpid()}"
    # Link with the host compiler against torch's runtime by full path, so the
    # library's NEEDED entry is the very libamdhip64.so torch loads.
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, "-Wl,--no-undefined",
           os.path.join(tlib, "libamdhip64.so"), os.path.join(tlib, "libhiprtc.so"),
           f"-Wl,-rpath,{tlib}", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
