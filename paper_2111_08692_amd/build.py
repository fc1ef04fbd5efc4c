"""Build the HIP library ``libutfgpu.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libutfgpu.so")
KERNEL_SOURCES = ["utf8_kernels.hip", "utf16_kernels.hip"]   # built once per tile geometry
API_SOURCE = "api.cpp"
ARCH = os.environ.get("UTFGPU_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere (they are not needed here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def geometries() -> list:
    """(namespace, waves, rows) of every line of csrc/geometries.def."""
    text = open(os.path.join(CSRC, "geometries.def")).read()
    return [(m.group(1), int(m.group(2)), int(m.group(3)))
            for m in re.finditer(r"^UTF_GEOMETRY\((\w+),\s*(\d+),\s*(\d+)\)", text, re.M)]


def build(verbose: bool = False) -> str:
    """Compile every source into ``libutfgpu.so`` (always recompiles): the
    kernel files once per tile geometry, in parallel, then the C ABI layer
    and the link."""
    objdir = tempfile.mkdtemp(prefix="utfgpu_build_")
    try:
        jobs = []
        for ns, waves, rows in geometries():
            for src in KERNEL_SOURCES:
                obj = os.path.join(objdir, f"{os.path.splitext(src)[0]}_{ns}.o")
                defs = [f"-DUTF_GEOM={ns}", f"-DUTF_WAVES={waves}", f"-DUTF_ROWS={rows}"]
                jobs.append([hipcc()] + FLAGS + defs + ["-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj])
        api_obj = os.path.join(objdir, "api.o")
        jobs.append([hipcc()] + FLAGS + ["-c", "-x", "hip", os.path.join(CSRC, API_SOURCE), "-o", api_obj])
        objs = [j[-1] for j in jobs]
        par = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        running = []
        for cmd in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append(subprocess.Popen(cmd))
            while len(running) >= par:
                _wait_one(running)
        while running:
            _wait_one(running)
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


def _wait_one(running: list) -> None:
    p = running.pop(0)
    if p.wait() != 0:
        for q in running:
            q.wait()
        raise subprocess.CalledProcessError(p.returncode, p.args)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
