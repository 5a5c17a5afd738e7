"""Builds libsv.so (the HIP library behind include/sv.h) for gfx950, in-tree.

Every .hip file under csrc/ is compiled to an object with hipcc in parallel,
then linked into paper_1801_01037_amd/libsv.so. Packed-FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsv.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
ARCH = "gfx950"

# -simplifycfg-sink-common=false: sinking the common code of switch arms into
# pointer selects over register arrays forces those arrays into scratch.
CFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-simplifycfg-sink-common=false",
          "-I", os.path.join(os.path.dirname(HERE), "include"), "-I", BUILD]


def _write_jit_sources() -> None:
    """The text of the headers a pass compiled at run time includes, as C
    string constants (jit_src.inc, included by jit.hip)."""
    out = []
    for var, name in (("kTileHSrc", "tile.h"), ("kTileDevHSrc", "tile_dev.h")):
        with open(os.path.join(CSRC, name)) as f:
            text = f.read()
        if ")SVJIT\"" in text:
            raise RuntimeError(f"{name} contains the raw-string delimiter")
        out.append(f'static const char {var}[] = R"SVJIT({text})SVJIT";\n')
    path = os.path.join(BUILD, "jit_src.inc")
    new = "".join(out)
    if not os.path.exists(path) or open(path).read() != new:
        with open(path, "w") as f:
            f.write(new)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature"
    warn = "\n".join(ln for ln in r.stderr.splitlines() if noise not in ln)
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _write_jit_sources()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L", os.path.join(ROCM, "lib"), "-lhiprtc"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
