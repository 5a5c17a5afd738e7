"""Shared helpers of the GPU tests: tolerances and state transfer."""
import contextlib
import math
import os

import numpy as np

import paper_1801_01037_amd as sv

U32 = 2.0 ** -24
C128_MAX_ABS = 1e-12


def c64_rel_tol(n_gates: int) -> float:
    """Relative 2-norm error bound stated for complex64 results: 8 sqrt(G) u32,
    G the number of gates applied (at least one)."""
    return 8.0 * math.sqrt(max(n_gates, 1)) * U32


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(got.astype(np.complex128) - ref) / np.linalg.norm(ref))


def max_abs(got: np.ndarray, ref: np.ndarray) -> float:
    return float(np.max(np.abs(got.astype(np.complex128) - ref)))


def assert_close(got: np.ndarray, ref: np.ndarray, dtype: int, n_gates: int, what=""):
    if dtype == sv.SV_C128:
        err = max_abs(got, ref)
        assert err <= C128_MAX_ABS, f"{what}: max-abs {err:.3e} > {C128_MAX_ABS:.0e}"
    else:
        err = rel_err(got, ref)
        tol = c64_rel_tol(n_gates)
        assert err <= tol, f"{what}: rel 2-norm {err:.3e} > {tol:.3e} (G={n_gates})"


def state_from_host(n: int, dtype: int, host: np.ndarray) -> int:
    """A library-owned state holding `host` (rounded to the state dtype)."""
    h = sv.sv_create(n, dtype)
    sv.sv_copy_in(h, host)
    return h


def rounded(host: np.ndarray, dtype: int) -> np.ndarray:
    """`host` as the GPU state stores it, back in complex128."""
    want = np.complex64 if dtype == sv.SV_C64 else np.complex128
    return host.astype(want).astype(np.complex128)


DTYPES = [sv.SV_C128, sv.SV_C64]
DTYPE_IDS = ["c128", "c64"]


@contextlib.contextmanager
def oracle_threads(k: int = 0):
    """Runs the oracle on k host threads (default: the host's cores, at most
    16) for the block, then back on one. The threaded build gives the same
    bits as the single-threaded one (pinned in tests/test_oracle.py)."""
    import oracle
    used = oracle.set_threads(k or min(16, os.cpu_count() or 1))
    try:
        yield used
    finally:
        oracle.set_threads(1)


# Sizes at which a state is larger than the last-level cache (streamed with the
# nontemporal hint) and each tile pass has more tiles than resident
# work-groups: (n, dtype) with 512 MiB states.
STREAMING = [(25, sv.SV_C128), (26, sv.SV_C64)]
STREAMING_IDS = ["25-c128", "26-c64"]
