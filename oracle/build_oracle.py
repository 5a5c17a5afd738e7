"""Builds the oracle's C libraries from sv_oracle.c with gcc (no HIP, no GPU).

liboracle.so      the reference build, single-threaded;
liboracle_omp.so  the same source with -fopenmp: the loops of one gate are
                  shared among threads (same bits as the reference build).

-ffp-contract=off keeps every multiply and add a separately rounded IEEE
operation; -O2 without -ffast-math keeps the evaluation order as written.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def _gcc(out: str, extra: list, verbose: bool) -> str:
    cmd = ["gcc", *_FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    _gcc(LIB_OMP, ["-fopenmp"], verbose)
    return _gcc(LIB, [], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
