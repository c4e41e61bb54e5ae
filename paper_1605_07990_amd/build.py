"""Build libim.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
LIB = HERE / "libim.so"
SOURCES = ["api.hip", "graph.hip", "sample.hip", "cover.hip", "engine.hip"]
# measurement helper (random-gather bandwidth probe), a library of its own
PROBE_LIB = HERE / "libimprobe.so"
PROBE_SOURCES = ["gather_probe.hip"]
ARCH = os.environ.get("IM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(path).exists():
        raise RuntimeError("hipcc not found: cannot build the HIP library")
    return path


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # keep packed FP32 instructions out of generated device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> Path:
    """Compile every source to an object, then link libim.so and the probe
    library (always rebuilds)."""
    _build_lib(SOURCES, LIB, verbose)
    _build_lib(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


def _build_lib(sources, lib: Path, verbose: bool) -> Path:
    objdir = HERE / "_build"
    objdir.mkdir(exist_ok=True)
    objs = []
    procs = []
    for src in sources:
        obj = objdir / (Path(src).stem + ".o")
        cmd = [hipcc(), *flags(), "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(str(obj))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(f"--- {src} ---\n{out}")
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError("HIP build failed:\n" + "\n".join(failed))
    tmp = str(lib) + ".tmp"
    subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
