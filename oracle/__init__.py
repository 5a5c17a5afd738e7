"""CPU complex128 oracle -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the smoke check in `__graft_entry__` and the CPU-baseline leg
of `bench.py` may import this package. The GPU library
(`paper_1801_01037_amd`) never imports it and shares no code with it; the only
thing both sides read is the serialized gate list from `qcircuits`.

Two tiers:
  * stride tier (`sv_oracle.c`, plain C): the paper's Algorithm 1 loops, gate
    by gate, at any n that fits host memory;
  * brute-force tier (`oracle.dense`, numpy): dense Kronecker-product
    operators for n <= 10 (the paper's direct approach).
Threads: `set_threads(k)` switches to the OpenMP build of the same C source
for k > 1 (the loops of each gate shared among k threads, the same bits as
the single-threaded reference build, which is the default).
Closed forms used as pins or as sampled references at large n:
  * `qft_basis_amplitude` (QFT of |x>), `product_state_amplitude` (circuits
    of one-qubit gates only, equation circuit-level), `uniform_amplitude`
    (H on every qubit of |0...0>).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None


def load(path: str):
    """Opens a built oracle library and declares its C signatures."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_init_basis.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
    L.orc_apply_1q.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
    L.orc_apply_ctrl.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    L.orc_apply_cphase.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double]
    L.orc_apply_mcu.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, dp]
    L.orc_apply_unitary.argtypes = [dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.c_int, dp]
    L.orc_apply_unitary.restype = ctypes.c_int
    L.orc_run_circuit.argtypes = [dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
    L.orc_run_circuit.restype = ctypes.c_int
    L.orc_probs.argtypes = [dp, ctypes.c_uint64, ctypes.c_uint64, dp]
    L.orc_norm.argtypes = [dp, ctypes.c_int]
    L.orc_norm.restype = ctypes.c_double
    L.orc_qft_basis_amplitude.argtypes = [ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_uint64, dp]
    L.orc_threads.argtypes = [ctypes.c_int]
    L.orc_threads.restype = ctypes.c_int
    return L


_ref = None
_omp = None


def _built(path):
    if not os.path.exists(path):
        build_oracle.build()
    return load(path)


def lib():
    """The library the functions below call (the single-threaded reference
    build unless set_threads chose the OpenMP one)."""
    global _lib, _ref
    if _lib is None:
        if _ref is None:
            _ref = _built(build_oracle.LIB)
        _lib = _ref
    return _lib


def set_threads(k: int) -> int:
    """k <= 1: the single-threaded reference build; k > 1: the OpenMP build
    with k threads. Returns the number of threads in effect."""
    global _lib, _ref, _omp
    if k <= 1:
        if _ref is None:
            _ref = _built(build_oracle.LIB)
        _lib = _ref
        return 1
    if _omp is None:
        _omp = _built(build_oracle.LIB_OMP)
    _lib = _omp
    return int(_omp.orc_threads(int(k)))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_state(psi: np.ndarray) -> int:
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous:
        raise TypeError("oracle states are C-contiguous complex128 arrays")
    n = int(psi.size).bit_length() - 1
    if psi.size != 1 << n:
        raise ValueError("state length must be a power of two")
    return n


def basis_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_basis(_dp(psi.view(np.float64)), n, x)
    return psi


def apply_1q(psi: np.ndarray, t: int, m) -> None:
    n = _check_state(psi)
    m = np.ascontiguousarray(m, dtype=np.float64)
    lib().orc_apply_1q(_dp(psi.view(np.float64)), n, t, _dp(m))


def apply_ctrl(psi: np.ndarray, c: int, t: int, m) -> None:
    n = _check_state(psi)
    m = np.ascontiguousarray(m, dtype=np.float64)
    lib().orc_apply_ctrl(_dp(psi.view(np.float64)), n, c, t, _dp(m))


def apply_mcu(psi: np.ndarray, controls, t: int, m) -> None:
    """2x2 gate on qubit t, applied where every qubit in `controls` is 1."""
    n = _check_state(psi)
    mask = 0
    for c in controls:
        mask |= 1 << int(c)
    m = np.ascontiguousarray(m, dtype=np.float64)
    lib().orc_apply_mcu(_dp(psi.view(np.float64)), n, mask, t, _dp(m))


def apply_unitary(psi: np.ndarray, qubits, u) -> None:
    """General gate: the 2^k x 2^k complex matrix u on qubits (q_0, ...,
    q_{k-1}), q_0 the least significant bit of the local index."""
    n = _check_state(psi)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    k = len(q)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    if u.shape != (1 << k, 1 << k):
        raise ValueError("u must be 2^k x 2^k")
    rc = lib().orc_apply_unitary(_dp(psi.view(np.float64)), n,
                                 q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), k,
                                 _dp(u.view(np.float64)))
    if rc != 0:
        raise ValueError("bad qubits for apply_unitary")


def apply_cphase(psi: np.ndarray, c: int, t: int, theta: float) -> None:
    n = _check_state(psi)
    lib().orc_apply_cphase(_dp(psi.view(np.float64)), n, c, t, float(theta))


def run_circuit(psi: np.ndarray, gates: np.ndarray, mats=None) -> None:
    """Applies a gate list (qcircuits.GATE_DTYPE records) in place, in order.
    General-gate records (kind 4) take their matrix from the side table
    `mats` (one row of 2048 doubles per matrix) and are applied by
    apply_unitary; runs of the other records by the C loop."""
    n = _check_state(psi)
    gates = np.ascontiguousarray(gates)
    general = np.flatnonzero(gates["kind"] == 4) if len(gates) else np.zeros(0, int)
    start = 0
    for i in list(general) + [len(gates)]:
        if i > start:
            part = np.ascontiguousarray(gates[start:i])
            rc = lib().orc_run_circuit(_dp(psi.view(np.float64)), n, part.ctypes.data, len(part))
            if rc != 0:
                raise ValueError("malformed gate record")
        if i < len(gates):
            g = gates[i]
            k = int(g["control"])
            packed = int(np.array(g["flags"], dtype=np.int32).view(np.uint32))
            qubits = [(packed >> (6 * j)) & 63 for j in range(k)]
            d = 1 << k
            row = np.asarray(mats[int(g["target"])], dtype=np.float64)[:2 * d * d]
            apply_unitary(psi, qubits, row.view(np.complex128).reshape(d, d))
        start = i + 1


def simulate(n: int, gates: np.ndarray, x: int = 0, mats=None) -> np.ndarray:
    psi = basis_state(n, x)
    run_circuit(psi, gates, mats)
    return psi


def probs(psi: np.ndarray, first: int = 0, count: int | None = None) -> np.ndarray:
    if count is None:
        count = psi.size - first
    out = np.empty(count, dtype=np.float64)
    lib().orc_probs(_dp(psi.view(np.float64)), first, count, _dp(out))
    return out


def norm(psi: np.ndarray) -> float:
    n = _check_state(psi)
    return float(lib().orc_norm(_dp(psi.view(np.float64)), n))


def qft_basis_amplitude(n: int, x: int, index: int) -> complex:
    out = np.empty(2)
    lib().orc_qft_basis_amplitude(n, x, index, _dp(out))
    return complex(out[0], out[1])


def qft_basis_amplitudes(n: int, x: int, indices) -> np.ndarray:
    return np.array([qft_basis_amplitude(n, x, int(i)) for i in indices])


def qubit_vectors(n: int, gates: np.ndarray, x: int = 0) -> np.ndarray:
    """For a circuit of one-qubit gates only: each qubit's own 2-vector after
    its gates, starting from bit q of |x> (the product-state rule: a tensor
    product of gates acts factor by factor, equation circuit-level)."""
    v = np.zeros((n, 2), dtype=np.complex128)
    for q in range(n):
        v[q, (x >> q) & 1] = 1.0
    for g in gates:
        if int(g["kind"]) != 0:
            raise ValueError("product-state rule needs one-qubit gates only")
        t = int(g["target"])
        m = g["m"]
        a, b = v[t]
        v[t, 0] = complex(m[0], m[1]) * a + complex(m[2], m[3]) * b
        v[t, 1] = complex(m[4], m[5]) * a + complex(m[6], m[7]) * b
    return v


def product_state_amplitude(vectors: np.ndarray, index: int) -> complex:
    """alpha_i = prod_q v_q[bit q of i]."""
    amp = 1.0 + 0.0j
    for q in range(vectors.shape[0]):
        amp *= vectors[q, (index >> q) & 1]
    return amp


def sample_indices(psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Measurement by inverting the CDF (the measurement of section Quantum
    Circuits: index j with probability |alpha_j|^2 / norm): for each u in
    [0, 1), the first j with CDF(j) > u * norm, CDF the running FP64 sum of
    |alpha|^2 in index order and norm its last entry. A u whose product with
    the norm is not below every CDF value (only by rounding) gets the last j
    of non-zero probability."""
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    cdf = np.cumsum(p)
    idx = np.searchsorted(cdf, np.asarray(u, dtype=np.float64) * cdf[-1], side="right")
    nz = np.flatnonzero(p)
    last = int(nz[-1]) if len(nz) else 0
    return np.where(idx >= len(p), last, idx).astype(np.uint64)


def uniform_amplitude(n: int) -> float:
    """Every amplitude of H on each qubit of |0...0>: 2^(-n/2)."""
    return 2.0 ** (-n / 2)
