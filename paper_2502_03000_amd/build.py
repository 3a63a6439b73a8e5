"""Builds the gfx950 shared library libhexla.so in-tree.

Kernels (*.hip) are compiled by hipcc for gfx950 with packed FP32 instructions
disabled; host sources (*.cpp) by the host C++ compiler against the HIP
runtime headers. Objects go to _build/, the library to _lib/.

    python -m paper_2502_03000_amd.build [-v]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libhexla.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-Wall", "-Wno-unused-result"]


def _hipcc() -> str:
    cand = os.path.join(ROCM, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def _torch_lib():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:  # noqa: BLE001
        pass
    return None


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source (always: a stale library is never reused) and
    links _lib/libhexla.so. Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    incs = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    cmds = []
    for src in sources():
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        path = os.path.join(CSRC, src)
        if src.endswith(".hip"):
            cmds.append([_hipcc(), *HIP_FLAGS, *incs, "-c", path, "-o", obj])
        else:
            cmds.append(["g++", *HOST_FLAGS, *incs, f"-I{ROCM}/include", "-c", path, "-o", obj])
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(lambda c: _run(c, verbose), cmds):
            if verbose and out.strip():
                print(out)
    objs = [os.path.join(BUILD, s.rsplit(".", 1)[0] + ".o") for s in sources()]
    tmp = LIB + ".tmp"
    # Prefer the HIP runtime bundled with torch (the process's torch uses it
    # for device memory and streams); fall back to the system ROCm.
    rpaths = [p for p in (_torch_lib(), f"{ROCM}/lib") if p]
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64", "-lhiprtc", *[f"-Wl,-rpath,{p}" for p in rpaths]], verbose)
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
