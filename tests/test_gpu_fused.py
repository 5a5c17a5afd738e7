"""GPU parity of the fused tile passes (SV_FUSE) against the CPU oracle.

Mixed random circuits exercise every op kind of a pass (general 2x2, X,
controlled 2x2 with controls inside and outside the tile, controlled phases
and one-qubit phases held back and merged into diagonal ops) at sizes below,
at and above one tile, plus the degenerate one- and two-qubit registers.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, STREAMING, STREAMING_IDS, assert_close
from tests.gpu_helpers import oracle_threads, rounded, state_from_host
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 12, 13, 14, 17, 20])
def test_mixed_circuit_fused(dtype, n):
    g = mixed_circuit(n, 400, 7 * n + 1)
    psi0 = rounded(qc.random_state(n, 300 + n), dtype)
    ref = psi0.copy()
    oracle.run_circuit(ref, g)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"fused mixed n={n}")


@pytest.mark.parametrize("n,dtype", STREAMING, ids=STREAMING_IDS)
def test_mixed_circuit_fused_streaming_sizes(n, dtype):
    """States past the last-level cache (tile loads and stores with the
    nontemporal hint) and many tiles per work-group (LDS slots reused from
    tile to tile), element by element against the oracle."""
    g = mixed_circuit(n, 400, 7 * n + 1)
    psi0 = rounded(qc.random_state(n, 300 + n), dtype)
    ref = psi0.copy()
    with oracle_threads():
        oracle.run_circuit(ref, g)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"fused mixed n={n}")


@pytest.mark.parametrize("n,dtype", STREAMING, ids=STREAMING_IDS)
def test_layers_qft_fused_streaming_sizes(n, dtype):
    """The benchmark's circuit kinds (layers, then the QFT) at streaming sizes."""
    g = np.concatenate([qc.layer_circuit(n, 6, n), qc.qft_circuit(n)])
    x = qc.random_basis_index(n, 3)
    with oracle_threads():
        ref = oracle.simulate(n, g, x)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_reset(h, x)
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"layers+qft fused n={n}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_layers_then_qft_16_qubits_fused(dtype):
    n = 16
    g = qc.workload_layers_qft(n, 100, 0)
    ref = oracle.simulate(n, g)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
        nrm = sv.sv_norm(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), "layers+qft fused")
    assert abs(nrm - 1.0) <= (1e-12 if dtype == sv.SV_C128 else 1e-5)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [4, 13, 18])
def test_qft_fused_matches_closed_form(dtype, n):
    for x in (0, 1, qc.random_basis_index(n, n)):
        h = sv.sv_create(n, dtype)
        try:
            sv.sv_reset(h, x)
            sv.sv_run_circuit(h, qc.qft_circuit(n), sv.SV_FUSE)
            got = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        ref = oracle.qft_basis_amplitudes(n, x, range(1 << n))
        assert_close(got, ref, dtype, n * (n + 1) // 2, f"qft n={n} x={x}")


def test_fused_results_are_bitwise_repeatable():
    n = 15
    g = mixed_circuit(n, 300, 5)
    outs = []
    for _ in range(2):
        h = sv.sv_create(n, sv.SV_C128)
        try:
            sv.sv_run_circuit(h, g, sv.SV_FUSE)
            outs.append(sv.sv_copy_out(h))
        finally:
            sv.sv_destroy(h)
    assert np.array_equal(outs[0], outs[1])


def test_fused_and_per_gate_calls_interleave():
    """Fused runs, per-gate calls and resets on one handle, in one stream."""
    n = 14
    g1 = mixed_circuit(n, 120, 1)
    g2 = mixed_circuit(n, 120, 2)
    ref = oracle.simulate(n, g1, 3)
    oracle.apply_1q(ref, 5, qc.H_MATRIX)
    oracle.run_circuit(ref, g2)
    h = sv.sv_create(n, sv.SV_C128)
    try:
        sv.sv_reset(h, 3)
        sv.sv_run_circuit(h, g1, sv.SV_FUSE)
        sv.sv_apply_1q(h, 5, qc.H_MATRIX)
        sv.sv_run_circuit(h, g2, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, sv.SV_C128, 241, "interleaved")
