"""GPU parity of gates with several controls (sv_apply_mcu, SV_G_MCU records)
against the CPU oracle, through the C ABI.

Control masks cover every layout of the pair kernel: a complex64 control on
bit 0 (odd amplitudes of a 16-byte chunk), a complex64 target on bit 0 (both
amplitudes in one chunk), controls below and above the target, many controls.
The Toffoli truth table is checked bit for bit.
"""
import math

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
def test_toffoli_truth_table(dtype):
    for t in range(3):
        c = [q for q in range(3) if q != t]
        for x in range(8):
            h = sv.sv_create(3, dtype)
            try:
                sv.sv_reset(h, x)
                sv.sv_apply_mcu(h, c, t, qc.X_MATRIX)
                got = sv.sv_copy_out(h)
            finally:
                sv.sv_destroy(h)
            both = (x >> c[0]) & 1 and (x >> c[1]) & 1
            assert np.array_equal(got, oracle.basis_state(3, x ^ (1 << t) if both else x)), (t, x)


CASES = [((1,), 0), ((0,), 5), ((0, 1), 2), ((0, 3), 1), ((2, 7), 0), ((0, 5, 9), 11),
         ((1, 2, 3, 4), 10), ((6, 8, 10, 11), 0), ((0, 1, 2, 3, 4, 5), 6)]


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_mcu_matches_oracle(dtype):
    n = 12
    psi0 = rounded(qc.random_state(n, 4242), dtype)
    mats = qc.haar_su2(99, len(CASES))
    ph = 0.7
    diag = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, math.cos(ph), math.sin(ph))
    for (controls, t), u in zip(CASES, mats):
        for m in (u, qc.X_MATRIX, diag):          # pair, exchange and phase kernels
            h = state_from_host(n, dtype, psi0)
            try:
                sv.sv_apply_mcu(h, controls, t, m)
                got = sv.sv_copy_out(h)
            finally:
                sv.sv_destroy(h)
            ref = psi0.copy()
            oracle.apply_mcu(ref, controls, t, m)
            assert_close(got, ref, dtype, 1, f"controls {controls} target {t}")
            if m is qc.X_MATRIX:                   # an exchange is exact
                assert np.array_equal(got, ref), (controls, t)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("flags", [0, sv.SV_FUSE, sv.SV_FUSE_DENSE], ids=["pergate", "fuse", "dense"])
def test_circuit_with_toffolis_matches_oracle(dtype, flags):
    """Records of several-control gates inside a circuit: in tile passes with
    the other gates (SV_FUSE), in dense blocks when they span at most five
    qubits (the last one, of five, does), gate by gate otherwise."""
    n = 14
    parts = [qc.layer_circuit(n, 3, 5)]
    for k in range(6):
        parts.append(qc.gate_mcu(((2 * k) % n, (2 * k + 3) % n), (2 * k + 7) % n, qc.X_MATRIX))
        parts.append(qc.layer_circuit(n, 1, 50 + k))
    parts.append(qc.gate_mcu((0, 1, 2, 13), 12, qc.haar_su2(7, 1)[0]))
    gates = np.concatenate(parts)
    psi0 = rounded(qc.random_state(n, 77), dtype)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, gates, flags)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    ref = psi0.copy()
    oracle.run_circuit(ref, gates)
    assert_close(got, ref, dtype, len(gates), f"flags {flags}")


def test_mcu_at_24_qubits():
    n = 24
    dtype = sv.SV_C128
    psi0 = qc.random_state(n, 24)
    u = qc.haar_su2(24, 1)[0]
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_apply_mcu(h, (0, 12, 23), 5, u)
        sv.sv_apply_mcu(h, (3, 4), 22, qc.X_MATRIX)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    ref = psi0.copy()
    oracle.apply_mcu(ref, (0, 12, 23), 5, u)
    oracle.apply_mcu(ref, (3, 4), 22, qc.X_MATRIX)
    assert_close(got, ref, dtype, 2, "24 qubits")


def test_mcu_rejects_bad_masks():
    h = sv.sv_create(5, sv.SV_C128)
    try:
        for controls, t in (((1, 2), 2), ((0, 5), 1), ((), 1)):
            with pytest.raises(sv.SVError) as e:
                sv.sv_apply_mcu(h, controls, t, qc.X_MATRIX)
            assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [3, 4, 6, 12, 13, 17, 20])
def test_several_controls_inside_fused_passes(dtype, n):
    """Mixed circuits with Toffolis and gates of up to four controls, fused:
    controls on register bits, on other tile bits and outside the tile, in
    relabelled and standard storage order, against the oracle."""
    g = mixed_circuit(n, 400, 13 * n + 2, mcu=True)
    psi0 = rounded(qc.random_state(n, 310 + n), dtype)
    ref = psi0.copy()
    oracle.run_circuit(ref, g)
    for flags in (sv.SV_FUSE, sv.SV_FUSE | sv.SV_NO_RELABEL, sv.SV_FUSE_DENSE):
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_run_circuit(h, g, flags)
            got = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        assert_close(got, ref, dtype, len(g), f"n={n} flags={flags}")


@pytest.mark.parametrize("n,dtype", STREAMING, ids=STREAMING_IDS)
def test_several_controls_inside_fused_passes_streaming_sizes(n, dtype):
    g = mixed_circuit(n, 300, 17 * n, mcu=True)
    psi0 = rounded(qc.random_state(n, 320 + n), dtype)
    ref = psi0.copy()
    with oracle_threads():
        oracle.run_circuit(ref, g)
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), f"n={n}")


def test_toffoli_circuits_batched():
    """Plans hold several-control gates, so circuits with Toffolis run in a
    batch (persistent launch, levels and the third stream) and give the
    bits of the circuit run alone."""
    dtype = sv.SV_C64
    specs = [(10, 1), (12, 2), (14, 3), (16, 4), (18, 5)]
    circuits = [np.concatenate([mixed_circuit(n, 200, s, mcu=True), qc.layer_circuit(n, 3, s)])
                for n, s in specs]
    states = [sv.sv_create(n, dtype) for n, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_persist(b, 4)
        sv.sv_batch_solo(b, 64)
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)
        outs = [sv.sv_copy_out(h) for h in states]
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    for (n, _), g, got in zip(specs, circuits, outs):
        h = sv.sv_create(n, dtype)
        try:
            sv.sv_run_circuit(h, g, sv.SV_FUSE)
            want = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        assert np.array_equal(got, want), n
        assert_close(got, oracle.simulate(n, g), dtype, len(g), f"batch n={n}")
