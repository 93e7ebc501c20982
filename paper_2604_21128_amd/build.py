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


def _object_key(src: str, flags) -> str:
    """Hash of a source, every header it may include and the flags (incremental builds)."""
    import hashlib
    h = hashlib.sha256(" ".join(flags).encode())
    headers = sorted(glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h")))
    for f in [src] + headers:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:24]


def build(verbose: bool = False, extra_flags=None, out: str = LIB,
          incremental: bool = False) -> str:
    """Compile all sources and link libqla.so (atomically replaced). Returns its path.
    incremental=True reuses objects under _build/ whose source, headers and flags are
    unchanged (a development shortcut; the default always compiles everything)."""
    cc = hipcc()
    flags = HIPCC_FLAGS + list(extra_flags or [])
    cache = os.path.join(ROOT, "_build")
    with tempfile.TemporaryDirectory(prefix="qla_build_") as tmp:
        objs = []
        procs = []
        for src in sources():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            final = obj
            if incremental:
                os.makedirs(cache, exist_ok=True)
                final = os.path.join(cache, os.path.basename(src) + "."
                                     + _object_key(src, flags) + ".o")
                if os.path.exists(final):
                    objs.append(final)
                    continue
            lang = ["-x", "hip"]
            cmd = [cc, *flags, "-I", INCLUDE, "-I", CSRC, *lang, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, obj, final, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                            stderr=subprocess.STDOUT, text=True)))
            objs.append(final)
        failed = []
        for src, obj, final, p in procs:
            log, _ = p.communicate()
            text = "\n".join(line for line in log.splitlines()
                             if "packed-fp32-ops" not in line)
            if p.returncode != 0:
                failed.append((src, text))
            else:
                if final != obj:
                    shutil.move(obj, final)
                if verbose and text.strip():
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
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
