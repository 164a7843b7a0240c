"""Builds libmbhip.so (the HIP kernels and the C ABI) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libmbhip.so")
OBJ = os.path.join(HERE, "_build")
# (source, extra flags, object name): the kernels are compiled in eighteen parts
# (FP32 and FP64, one-chunk and persistent tiles, exact and Cayley field step,
# general and block form of the density tables; the work-queue kernels)
SOURCES = [("kernels.hip", [f"-DMB_PART={i + 1}"], f"kernels_{i:02d}") for i in range(18)] + [
    ("scratch.hip", [], "scratch")] + [(f, [], f) for f in ("plan.cpp", "runtime.cpp", "tune.cpp", "abi.cpp", "server.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MB_OFFLOAD_ARCH", "gfx950")

COMMON = ["-std=c++17", "-O3", "-fPIC", "-ffp-contract=off", f"-I{INCLUDE}", f"-I{CSRC}"]
# packed FP32 instructions stay disabled in device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _deps(src: str):
    """Files an object depends on: the kernels on their own headers, the host
    sources on every header (they share the plan and engine structures)."""
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    heads += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    if src.endswith(".hip"):
        heads = [h for h in heads if os.path.basename(h) in ("engine.hpp", "launch.hpp", "scratch.hpp")]
    return [os.path.join(CSRC, src)] + heads


def _compile(item, incremental=False) -> str:
    src, extra, name = item
    obj = os.path.join(OBJ, name + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(map(os.path.getmtime, _deps(src))):
        return obj
    cmd = [HIPCC] + COMMON + DEVICE + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if not src.endswith(".hip"):
        cmd = [HIPCC] + COMMON + extra + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c",
                                          os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"compiling {src} failed")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (incremental: only objects older than their
    sources or headers) and links libmbhip.so."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda it: _compile(it, incremental), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libmbhip.so failed")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
