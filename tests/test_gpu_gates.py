"""GPU parity of the per-gate kernels against the CPU oracle, through the C ABI.

Inputs are seeded (qcircuits); the oracle gets the same input amplitudes as
the GPU state holds (rounded to complex64 for the c64 runs). Sizes span
several 16-byte chunks per block and the degenerate tiny registers (n = 1, 2).
"""
import math

import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close, rounded, state_from_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [1, 2, 3, 9, 16])
def test_reset_gives_basis_state(dtype, n):
    h = sv.sv_create(n, dtype)
    try:
        assert np.array_equal(sv.sv_copy_out(h), oracle.basis_state(n, 0))
        x = (1 << n) - 1 if n < 9 else 0x155 % (1 << n)
        sv.sv_reset(h, x)
        assert np.array_equal(sv.sv_copy_out(h), oracle.basis_state(n, x))
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [1, 2, 3, 11])
def test_one_qubit_gate_every_target(dtype, n):
    psi0 = rounded(qc.random_state(n, 1000 + n), dtype)
    mats = qc.haar_su2(n, n)
    for t in range(n):
        for m in (mats[t], qc.X_MATRIX, qc.H_MATRIX):
            h = state_from_host(n, dtype, psi0)
            try:
                sv.sv_apply_1q(h, t, m)
                got = sv.sv_copy_out(h)
            finally:
                sv.sv_destroy(h)
            ref = psi0.copy()
            oracle.apply_1q(ref, t, m)
            assert_close(got, ref, dtype, 1, f"n={n} t={t}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [2, 3, 7, 9])
def test_controlled_gate_every_pair(dtype, n):
    psi0 = rounded(qc.random_state(n, 2000 + n), dtype)
    mats = qc.haar_su2(77, n * n)
    phase = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, math.cos(0.3), math.sin(0.3))
    for c in range(n):
        for t in range(n):
            if c == t:
                continue
            for m in (mats[c * n + t], qc.X_MATRIX, phase):
                h = state_from_host(n, dtype, psi0)
                try:
                    sv.sv_apply_ctrl(h, c, t, m)
                    got = sv.sv_copy_out(h)
                finally:
                    sv.sv_destroy(h)
                ref = psi0.copy()
                oracle.apply_ctrl(ref, c, t, m)
                assert_close(got, ref, dtype, 1, f"c={c} t={t}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_cnot_is_exact_permutation(dtype):
    n = 10
    psi0 = rounded(qc.random_state(n, 31), dtype)
    for c, t in [(0, 1), (1, 0), (0, 9), (9, 0), (4, 5), (8, 2)]:
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_apply_ctrl(h, c, t, qc.X_MATRIX)
            got = sv.sv_copy_out(h).astype(np.complex128)
        finally:
            sv.sv_destroy(h)
        ref = psi0.copy()
        oracle.apply_ctrl(ref, c, t, qc.X_MATRIX)
        assert np.array_equal(got, ref), (c, t)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_controlled_phase(dtype):
    n = 9
    psi0 = rounded(qc.random_state(n, 41), dtype)
    cases = [(0, 1, math.pi / 2), (1, 0, 2 * math.pi / 2 ** 8), (0, 8, -1.25),
             (8, 3, 2 * math.pi / 2 ** 30), (4, 5, 3.0), (2, 7, math.pi)]
    for c, t, th in cases:
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_apply_cphase(h, c, t, th)
            got = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        ref = psi0.copy()
        oracle.apply_cphase(ref, c, t, th)
        assert_close(got, ref, dtype, 1, f"c={c} t={t} theta={th}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_layers_then_qft_16_qubits(dtype):
    """16 qubits from |0...0>: 100 random layers then a QFT (2486 gates)."""
    n = 16
    g = qc.workload_layers_qft(n, 100, 0)
    ref = oracle.simulate(n, g)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_run_circuit(h, g)
        got = sv.sv_copy_out(h)
        p = sv.sv_probs(h, 0, 1 << n)
        nrm = sv.sv_norm(h)
    finally:
        sv.sv_destroy(h)
    assert_close(got, ref, dtype, len(g), "layers+qft")
    pref = oracle.probs(ref)
    if dtype == sv.SV_C128:
        assert np.max(np.abs(p - pref)) <= 1e-12
        assert abs(nrm - oracle.norm(ref)) <= 1e-12
    else:
        assert abs(nrm - 1.0) <= 1e-5


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_probs_ranges_and_norm(dtype):
    n = 13
    psi0 = rounded(qc.random_state(n, 5), dtype)
    h = state_from_host(n, dtype, psi0)
    try:
        pref = oracle.probs(psi0)
        for first, count in [(0, 1 << n), (3, 1000), (1 << n, 0), ((1 << n) - 1, 1),
                             (4097, 3001)]:
            got = sv.sv_probs(h, first, count)
            assert got.shape == (count,)
            assert np.max(np.abs(got - pref[first:first + count]), initial=0) <= 1e-15
        a = sv.sv_norm(h)
        b = sv.sv_norm(h)
        assert a == b                       # fixed reduction tree: same bits
        assert abs(a - oracle.norm(psi0)) <= 1e-13
        with pytest.raises(sv.SVError):
            sv.sv_probs(h, 1, 1 << n)
    finally:
        sv.sv_destroy(h)


def test_errors_leave_state_untouched():
    n = 6
    psi0 = qc.random_state(n, 9)
    h = state_from_host(n, sv.SV_C128, psi0)
    try:
        bad = [
            lambda: sv.sv_apply_1q(h, n, qc.X_MATRIX),
            lambda: sv.sv_apply_1q(h, -1, qc.X_MATRIX),
            lambda: sv.sv_apply_ctrl(h, 2, 2, qc.X_MATRIX),
            lambda: sv.sv_apply_cphase(h, 0, n, 0.5),
            lambda: sv.sv_reset(h, 1 << n),
            lambda: sv.sv_run_circuit(h, np.concatenate([qc.gate_u(0, qc.H_MATRIX),
                                                         qc.gate_cnot(1, 1)])),
            lambda: sv.sv_apply_1q(h, 0, (float("nan"),) + qc.X_MATRIX[1:]),
        ]
        for fn in bad:
            with pytest.raises(sv.SVError) as ei:
                fn()
            assert ei.value.status == sv.SV_EINVAL
        assert np.array_equal(sv.sv_copy_out(h), psi0)
    finally:
        sv.sv_destroy(h)


def test_results_are_bitwise_repeatable():
    n = 14
    g = qc.layer_circuit(n, 6, 3)
    outs = []
    for _ in range(2):
        h = sv.sv_create(n, sv.SV_C128)
        try:
            sv.sv_run_circuit(h, g)
            outs.append(sv.sv_copy_out(h))
        finally:
            sv.sv_destroy(h)
    assert np.array_equal(outs[0], outs[1])


def test_torch_wrapped_state_matches_owned_state():
    import torch
    n = 12
    g = qc.layer_circuit(n, 4, 8)
    with sv.StateVector(n, sv.SV_C128) as st:
        st.run(g)
        torch.cuda.synchronize()
        a = st.tensor.cpu().numpy()
    ref = oracle.simulate(n, g)
    assert np.max(np.abs(a - ref)) <= 1e-12


@pytest.mark.parametrize("dtype,n", [(sv.SV_C128, 25), (sv.SV_C64, 26)], ids=["c128-25", "c64-26"])
def test_streamed_state_every_pair_layout(dtype, n):
    """A state past the last-level cache (512 MiB) takes the streaming
    accesses; targets whose pairs lie within one wave's 64 chunks take the
    lane exchange (unless a control inserted into the work index lies below
    the target), targets 16 MiB or more apart two or four pairs per thread,
    and controls inside a line are tested per amplitude, as are phases on
    bits inside a line. One sequence covers each, against the oracle."""
    def phase(theta):
        return (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, math.cos(theta), math.sin(theta))

    psi0 = rounded(qc.random_state(n, 2500 + n), dtype)
    mats = qc.haar_su2(2600 + n, 16)
    seq = [((), 0, mats[0]), ((), 1, mats[1]), ((), 2, mats[2]), ((), 3, mats[3]),
           ((), 4, mats[4]), ((), n - 4, mats[5]), ((), n - 1, mats[6]),
           ((0,), n - 1, qc.X_MATRIX), ((n - 1,), 0, mats[7]), ((2,), 1, mats[8]),
           ((0,), 3, mats[9]), ((1, n - 2), 3, mats[10]), ((0, 1, 2), n - 1, qc.X_MATRIX),
           ((3, 20), 0, qc.X_MATRIX), ((0, 5), 2, mats[11]),
           ((0,), n - 1, phase(0.3)), ((14,), 15, phase(0.5)), ((2,), 5, phase(0.7)),
           ((0, 1), 2, phase(1.1)), ((), 5, mats[12]), ((), 6, mats[13]), ((4,), 5, mats[14]),
           ((7,), 5, mats[15]), ((9, 1), 6, qc.X_MATRIX), ((), 7, mats[0]), ((), 9, mats[1]),
           ((), 10, mats[2]), ((8,), 7, mats[3]), ((6,), 8, mats[4]), ((12, 0), 9, mats[5])]
    h = state_from_host(n, dtype, psi0)
    try:
        for controls, t, m in seq:
            if controls:
                sv.sv_apply_mcu(h, controls, t, m)
            else:
                sv.sv_apply_1q(h, t, m)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    ref = psi0.copy()
    for controls, t, m in seq:
        if controls:
            oracle.apply_mcu(ref, controls, t, m)
        else:
            oracle.apply_1q(ref, t, m)
    assert_close(got, ref, dtype, len(seq), f"n={n}")
