"""GPU parity of the dense 5-qubit MFMA blocks (SV_FUSE_DENSE) against the
CPU oracle, and against the per-gate path at 30 qubits."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import C128_MAX_ABS, DTYPE_IDS, DTYPES, assert_close, c64_rel_tol
from tests.gpu_helpers import STREAMING, STREAMING_IDS, oracle_threads, rounded, state_from_host
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [5, 9, 10, 13, 16])
def test_mixed_circuit_dense(dtype, n):
    g = mixed_circuit(n, 300, 11 * n + 3)
    psi0 = rounded(qc.random_state(n, 700 + n), dtype)
    ref = psi0.copy()
    oracle.run_circuit(ref, g)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE_DENSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"dense mixed n={n}")


@pytest.mark.parametrize("n,dtype", STREAMING, ids=STREAMING_IDS)
def test_mixed_circuit_dense_streaming_sizes(n, dtype):
    """Dense blocks on states past the last-level cache (blocks with no qubit
    inside a 128-byte line stream with the nontemporal hint), against the
    oracle element by element."""
    g = mixed_circuit(n, 300, 11 * n + 3)
    psi0 = rounded(qc.random_state(n, 700 + n), dtype)
    ref = psi0.copy()
    with oracle_threads():
        oracle.run_circuit(ref, g)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE_DENSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"dense mixed n={n}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_layers_then_qft_16_qubits_dense(dtype):
    n = 16
    g = qc.workload_layers_qft(n, 100, 0)
    ref = oracle.simulate(n, g)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE_DENSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), "layers+qft dense")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_qft_dense_matches_closed_form(dtype):
    n = 14
    x = qc.random_basis_index(n, 77)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_reset(h, x)
        sv.sv_run_circuit(h, qc.qft_circuit(n), sv.SV_FUSE_DENSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    ref = oracle.qft_basis_amplitudes(n, x, range(1 << n))
    assert_close(got, ref, dtype, n * (n + 1) // 2, "qft dense")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_dense_against_per_gate_30_qubits(dtype):
    import torch
    g = qc.layer_circuit(30, 4, 21)
    with sv.StateVector(30, dtype) as a, sv.StateVector(30, dtype) as b:
        a.run(g, 0)
        b.run(g, sv.SV_FUSE_DENSE)
        torch.cuda.synchronize()
        if dtype == sv.SV_C128:
            err = (a.tensor - b.tensor).abs().max().item()
            assert err <= C128_MAX_ABS
        else:
            err = ((a.tensor - b.tensor).norm() / a.tensor.norm()).item()
            assert err <= 2 * c64_rel_tol(len(g))
