"""Brute-force tier of the oracle (TEST INFRASTRUCTURE, n <= 10).

Builds each gate's full 2^n x 2^n operator by Kronecker products and applies
it as one dense matrix-vector product, which is the paper's direct approach
(Direct Approach: applying a circuit level is the matrix-vector product
psi' = U psi, with U the tensor product of the per-qubit gates, equations
tensor-product-gates and circuit-level). This tier shares no code with the
stride tier in sv_oracle.c; agreement of the two pins both.

Index convention: qubit q is bit q of the amplitude index, so the operator of
Q on qubit t is I_{2^(n-1-t)} (x) Q (x) I_{2^t} (the most significant qubit is
the leftmost Kronecker factor). A controlled gate is
P0_c (x) I  +  P1_c (x) Q_t  (projectors on the control bit, identities
elsewhere), which acts with Q only where bit c is one (caption of Algorithm 1);
with several controls (the Toffoli gate of section Quantum Circuits is X with
two) the projectors of all of them multiply.
"""
from __future__ import annotations

import numpy as np

MAX_QUBITS = 10

_I2 = np.eye(2, dtype=np.complex128)
_P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
_P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def matrix_of(m) -> np.ndarray:
    """2x2 complex matrix from the 8 doubles q11, q12, q21, q22 as (re, im)."""
    m = np.asarray(m, dtype=np.float64)
    return (m[0::2] + 1j * m[1::2]).reshape(2, 2)


def _kron_chain(factors_by_qubit: dict, n: int) -> np.ndarray:
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):          # most significant qubit first
        out = np.kron(out, factors_by_qubit.get(q, _I2))
    return out


def operator_1q(n: int, t: int, q: np.ndarray) -> np.ndarray:
    return _kron_chain({t: q}, n)


def operator_ctrl(n: int, c: int, t: int, q: np.ndarray) -> np.ndarray:
    return _kron_chain({c: _P0}, n) + _kron_chain({c: _P1, t: q}, n)


def operator_mcu(n: int, controls, t: int, q: np.ndarray) -> np.ndarray:
    """Q on t where every control qubit is one: I + (P1 on each control) (x) (Q - I)_t."""
    factors = {int(c): _P1 for c in controls}
    factors[t] = q - _I2
    return np.eye(2 ** n, dtype=np.complex128) + _kron_chain(factors, n)


def operator_unitary(n: int, qubits, u: np.ndarray) -> np.ndarray:
    """The general gate u on (q_0, ..., q_{k-1}) as a sum of Kronecker chains:
    u = sum_{r,c} u[r, c] |r><c|, and |r><c| on k qubits is the product of the
    2x2 matrix units |r_m><c_m| on qubit q_m (r_m = bit m of r)."""
    k = len(qubits)
    out = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for r in range(2 ** k):
        for c in range(2 ** k):
            if u[r, c] == 0:
                continue
            factors = {}
            for m, q in enumerate(qubits):
                e = np.zeros((2, 2), dtype=np.complex128)
                e[(r >> m) & 1, (c >> m) & 1] = 1.0
                factors[int(q)] = e
            out += u[r, c] * _kron_chain(factors, n)
    return out


def operator_cphase(n: int, c: int, t: int, theta: float) -> np.ndarray:
    return operator_ctrl(n, c, t, np.diag([1.0, np.exp(1j * theta)]))


def _table_matrix(g, mats) -> np.ndarray:
    """A general gate's 2^k x 2^k matrix from its side-table row."""
    k = int(g["control"])
    d = 1 << k
    row = np.asarray(mats[int(g["target"])], dtype=np.float64)[:2 * d * d]
    return row.view(np.complex128).reshape(d, d)


def _record_qubits(g) -> list:
    packed = int(np.array(g["flags"], dtype=np.int32).view(np.uint32))
    return [(packed >> (6 * j)) & 63 for j in range(int(g["control"]))]


def gate_operator(n: int, g, mats=None) -> np.ndarray:
    kind, c, t = int(g["kind"]), int(g["control"]), int(g["target"])
    if kind == 4:   # general gate on the listed qubits, matrix from the side table
        return operator_unitary(n, _record_qubits(g), _table_matrix(g, mats))
    if kind == 0:
        return operator_1q(n, t, matrix_of(g["m"]))
    if kind == 1:
        return operator_ctrl(n, c, t, matrix_of(g["m"]))
    if kind == 2:
        return operator_cphase(n, c, t, float(g["m"][0]))
    if kind == 3:
        lo = int(np.array(g["control"], dtype=np.int32).view(np.uint32))
        hi = int(np.array(g["flags"], dtype=np.int32).view(np.uint32))
        mask = lo | (hi << 32)
        return operator_mcu(n, [q for q in range(n) if (mask >> q) & 1], t, matrix_of(g["m"]))
    raise ValueError(f"unknown gate kind {kind}")


def run_circuit(n: int, gates, psi0: np.ndarray, mats=None) -> np.ndarray:
    """psi = U_G ... U_1 psi0 with every U_g built densely (`mats`: the side
    table of general-gate records)."""
    if n > MAX_QUBITS:
        raise ValueError("the dense tier is for n <= 10")
    psi = np.array(psi0, dtype=np.complex128)
    for g in gates:
        psi = gate_operator(n, g, mats) @ psi
    return psi


def circuit_unitary(n: int, gates) -> np.ndarray:
    u = np.eye(2 ** n, dtype=np.complex128)
    for g in gates:
        u = gate_operator(n, g) @ u
    return u
