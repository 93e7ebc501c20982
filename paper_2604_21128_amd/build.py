"""Build the gfx950 QLA library (libqla.so) in-tree with hipcc.

`python -m paper_2604_21128_amd.build` (or `build()`) compiles every HIP/C++
source under csrc/ for gfx950 and links them into paper_2604_21128_amd/libqla.so.
It always recompiles, so a call after a source change is a real build check.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqla.so")
ARCH = os.environ.get("QLA_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
    # no packed-FP32 instructions: scalar and float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (ROCm is required to build libqla.so)")
    return path


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, extra_flags=None, out: str = LIB) -> str:
    """Compile all sources and link libqla.so (atomically replaced). Returns its path."""
    cc = hipcc()
    flags = HIPCC_FLAGS + list(extra_flags or [])
    with tempfile.TemporaryDirectory(prefix="qla_build_") as tmp:
        objs = []
        procs = []
        for src in sources():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
            cmd = [cc, *flags, "-I", INCLUDE, "-I", CSRC, *lang, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            log, _ = p.communicate()
            text = "\n".join(line for line in log.splitlines()
                             if "packed-fp32-ops" not in line)
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
            raise RuntimeError(f"hipcc failed:\n{msg}")
        tmp_lib = os.path.join(tmp, "libqla.so")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        staged = out + ".tmp"
        shutil.copyfile(tmp_lib, staged)
        os.replace(staged, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
