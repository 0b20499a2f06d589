"""Build the HIP library libtpf.so for gfx950 (in-tree, next to this file).

Every kernel is compiled with packed-FP32 instructions disabled; the host
code is plain C++17.  The translation units are compiled in parallel
and linked into one shared library exporting the C ABI of include/tpf.h.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtpf.so")
SOURCES = ["tpf_stage.hip", "tpf_poisson.hip", "tpf_host.hip", "tpf_batch.hip", "tpf_adjoint.hip",
           "tpf_implicit.hip"]
ARCH = os.environ.get("TPF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Wno-unused-result", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# debug builds only: clamp every stage-kernel neighbour index to the grid
# (the periodic offsets are checked cell by cell on the CPU by tests/index_check.cpp)
if os.environ.get("TPF_BOUNDS_CLAMP") == "1":
    CFLAGS.append("-DTPF_BOUNDS_CLAMP")


def source_hash() -> str:
    """16 hex digits over the library's sources (kernels, host code, header):
    built into the library so that caches keyed on it (the batch tuner's)
    are not reused across source changes."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    for f in files + [os.path.join("..", "..", "include", "tpf.h")]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC, *CFLAGS, f'-DTPF_SRC_HASH="{source_hash()}"', "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # hipcc's host pass reports the GPU-only target feature as unknown: harmless
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
