"""GPU parity of general gates on k qubits (sv_apply_unitary) against the CPU
oracle, through the C ABI.

k >= 2 on n >= 9 qubits runs as one dense 5-qubit block on the matrix cores
(the gate padded with the identity on unused high qubits); smaller registers
use the small-register kernel; k = 1 is the pair update. Qubit lists cover
low qubits inside one 128-byte line, high qubits, unsorted orders and the
padding choices. Tolerances: complex128 1e-12 max-abs; complex64 the stated
8 sqrt(G) 2^-24 relative bound with G = 2^k, the number of terms summed into
each output.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close, rounded, state_from_host

pytestmark = pytest.mark.gpu

QUBITS = {
    1: [(0,), (4,)],
    2: [(0, 1), (1, 0), (3, 7), (8, 2)],
    3: [(0, 1, 2), (7, 0, 4), (2, 8, 5)],
    4: [(0, 1, 2, 3), (8, 1, 6, 3), (4, 2, 7, 0)],
    5: [(0, 1, 2, 3, 4), (8, 0, 5, 2, 6), (4, 3, 2, 1, 0)],
}


def _apply(n, dtype, psi0, qubits, u):
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_apply_unitary(h, qubits, u)
        return sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [5, 8, 9, 12, 17])
def test_unitary_matches_oracle(dtype, n):
    psi0 = rounded(qc.random_state(n, 700 + n), dtype)
    for k, lists in QUBITS.items():
        for qubits in lists:
            if max(qubits) >= n:
                continue
            u = qc.random_unitary(k, 10 * k + sum(qubits))
            ref = psi0.copy()
            oracle.apply_unitary(ref, qubits, u)
            got = _apply(n, dtype, psi0, qubits, u)
            assert_close(got, ref, dtype, 1 << k, f"n={n} qubits={qubits}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [6, 10])
def test_identity_is_exact(dtype, n):
    psi0 = rounded(qc.random_state(n, 5), dtype)
    for qubits in ((0, 1), (1, 3, 0, 5, 2)):
        got = _apply(n, dtype, psi0, qubits, np.eye(1 << len(qubits)))
        assert np.array_equal(got, psi0), qubits


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_tensor_product_equals_two_one_qubit_gates(dtype):
    n = 14
    ma, mb = qc.haar_su2(21, 2)
    A, B = qc.random_unitary(1, 3), qc.random_unitary(1, 4)
    psi0 = rounded(qc.random_state(n, 9), dtype)
    for a, b in ((0, 13), (6, 2)):
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_apply_1q(h, a, A.view(np.float64).ravel())
            sv.sv_apply_1q(h, b, B.view(np.float64).ravel())
            ref = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        got = _apply(n, dtype, psi0, (a, b), np.kron(B, A))
        assert_close(got, ref.astype(np.complex128), dtype, 4, f"({a}, {b})")


def test_unitary_then_inverse_at_22_qubits():
    n = 22
    psi0 = qc.random_state(n, 22)
    h = state_from_host(n, sv.SV_C128, psi0)
    try:
        for k, qubits in ((2, (21, 0)), (3, (5, 20, 11)), (5, (0, 3, 19, 7, 12))):
            u = qc.random_unitary(k, 500 + k)
            sv.sv_apply_unitary(h, qubits, u)
            ref = psi0.copy()
            oracle.apply_unitary(ref, qubits, u)
            got = sv.sv_copy_out(h)
            assert_close(got, ref, sv.SV_C128, 1, f"k={k}")
            sv.sv_apply_unitary(h, qubits, u.conj().T)
            assert_close(sv.sv_copy_out(h), psi0, sv.SV_C128, 2, f"k={k} inverse")
    finally:
        sv.sv_destroy(h)


def test_unitary_rejects_bad_arguments():
    h = sv.sv_create(6, sv.SV_C128)
    try:
        for qubits in ((1, 1), (6,), (-1, 2), (0, 1, 2, 3, 4, 5)):
            with pytest.raises(sv.SVError) as e:
                sv.sv_apply_unitary(h, qubits, np.eye(1 << len(qubits)))
            assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(h)
    h = sv.sv_create(2, sv.SV_C64)
    try:
        with pytest.raises(sv.SVError) as e:
            sv.sv_apply_unitary(h, (0, 1, 2), np.eye(8))
        assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(h)


def _general_circuit(n, seed):
    """Layers, a Toffoli and general gates on k = 1..5 qubits (list order
    mixed, low and high qubits), with their side table."""
    ks = [2, 3, 5, 1, 4, 2]
    mats = [qc.random_unitary(k, seed + 10 * k + j) for j, k in enumerate(ks)]
    rng = np.random.default_rng(seed)
    parts = [qc.layer_circuit(n, 2, seed)]
    for j, k in enumerate(ks):
        qs = rng.choice(n, size=k, replace=False)
        parts.append(qc.gate_unitary(qs, j))
        parts.append(qc.layer_circuit(n, 1, seed + j + 1))
    parts.append(qc.gate_mcu((0, n - 1), 1, qc.X_MATRIX))
    parts.append(qc.gate_unitary(list(range(n - 5, n)), 2))
    return np.concatenate(parts), qc.unitary_table(mats)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [6, 10, 16])
def test_circuits_with_general_gates(dtype, n):
    """SV_G_UNITARY records inside circuits (sv_run_circuit_ex): gate by gate,
    fused (generic and compiled passes) and dense, against the oracle."""
    g, tab = _general_circuit(n, 50 + n)
    psi0 = rounded(qc.random_state(n, 60 + n), dtype)
    ref = psi0.copy()
    oracle.run_circuit(ref, g, tab)
    # G: the gates applied, a general gate counting its 2^k terms
    G = int(sum(1 << int(x["control"]) if int(x["kind"]) == qc.G_UNITARY else 1 for x in g))
    for flags in (0, sv.SV_FUSE, sv.SV_FUSE | sv.SV_JIT, sv.SV_FUSE_DENSE):
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_run_circuit(h, g, flags, tab)
            got = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        assert_close(got, ref, dtype, G, f"n={n} flags={flags}")


def test_general_gate_records_are_checked():
    n = 8
    g, tab = _general_circuit(n, 3)
    h = sv.sv_create(n, sv.SV_C128)
    try:
        sv.sv_reset(h, 9)
        before = sv.sv_copy_out(h)
        bad = [g.copy() for _ in range(3)]
        bad[0][len(g) // 2] = qc.gate_unitary([1, 1], 0)[0]      # a qubit twice
        bad[1][len(g) // 2] = qc.gate_unitary([1, 2], 99)[0]     # matrix index past the table
        bad[2][len(g) // 2] = qc.gate_unitary([1, 8], 0)[0]      # qubit outside the register
        for b in bad:
            with pytest.raises(sv.SVError) as e:
                sv.sv_run_circuit(h, b, sv.SV_FUSE, tab)
            assert e.value.status == sv.SV_EINVAL
        with pytest.raises(sv.SVError) as e:                     # no table at all
            sv.sv_run_circuit(h, g, sv.SV_FUSE)
        assert e.value.status == sv.SV_EINVAL
        with pytest.raises(sv.SVError) as e:
            sv.sv_run_circuit(h, g, sv.SV_FUSE | sv.SV_GRAPH, tab)
        assert e.value.status == sv.SV_EUNSUPPORTED
        assert np.array_equal(sv.sv_copy_out(h), before)          # nothing ran
    finally:
        sv.sv_destroy(h)
