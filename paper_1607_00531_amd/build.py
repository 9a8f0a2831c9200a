"""Build the HIP library libepi.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Each source is compiled to an object in parallel (objects under _build/, not committed),
then the objects are linked into paper_1607_00531_amd/libepi.so."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libepi.so")
OBJDIR = os.path.join(ROOT, "_build", "epi")
SOURCES = ["epi_api.hip", "epi_line.hip", "epi_vec.hip", "epi_dct.hip", "epi_batch.hip",
           "epi_serve.hip", "epi_multilevel.hip", "epi_noalloc.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libepi.so)")


def flags() -> list:
    return [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
        # packed float32 VALU forms are disabled for all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fvisibility=hidden",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


def build_command(out: str = LIB) -> list:
    """The whole library in one hipcc invocation (same flags as the parallel build)."""
    return [hipcc(), *flags(), "-shared", *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), *flags(), "-c", os.path.join(CSRC, src), "-o", obj]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link paper_1607_00531_amd/libepi.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))

    def run(cmd):
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(run, [compile_command(s, o) for s, o in zip(SOURCES, objs)]))
    for src, res in zip(SOURCES, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed compiling {src}")
        if verbose:
            sys.stdout.write(res.stdout)
    tmp = LIB + ".tmp"
    res = run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libepi.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
