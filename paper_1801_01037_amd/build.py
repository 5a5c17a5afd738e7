"""Builds libsv.so (the HIP library behind include/sv.h) for gfx950, in-tree.

Every .hip file under csrc/ is compiled to an object with hipcc in parallel,
then linked into paper_1801_01037_amd/libsv.so. Packed-FP32 instructions are
disabled for all device code.

`--host-asan` builds a copy whose host code (the planner, the C ABI, the
code generator of compiled passes) carries AddressSanitizer, into
_build_asan/libsv_asan.so; device code is built as usual. It is for checking
the host code on the CPU (tests/run_host_asan.py), never for GPU runs.
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
BUILD_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(BUILD_ASAN, "libsv_asan.so")
# AddressSanitizer on the host pass only (each flag behind -Xarch_host).
ASAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
ASAN_LINK = ["-Xarch_host", "-fsanitize=address"]
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


def _compile(src: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature"
    warn = "\n".join(ln for ln in r.stderr.splitlines() if noise not in ln)
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False, host_asan: bool = False) -> str:
    out_dir, lib, extra, link = ((BUILD_ASAN, LIB_ASAN, ASAN_FLAGS, ASAN_LINK) if host_asan
                                 else (BUILD, LIB, [], []))
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(out_dir, exist_ok=True)
    _write_jit_sources()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link, "-o", tmp, *objs,
           "-L", os.path.join(ROCM, "lib"), "-lhiprtc"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, lib)
    if verbose:
        print(lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, host_asan="--host-asan" in sys.argv[1:])
