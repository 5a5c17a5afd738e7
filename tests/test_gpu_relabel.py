"""GPU parity of relabelled tile passes (SV_FUSE, the paper's non-sequential
storage) against the CPU oracle, and against the same circuit planned in the
standard storage order (SV_FUSE | SV_NO_RELABEL).

Each case first checks on the host that the planner keeps the relabelled
plan (fewer passes), so the relabelled store really runs. The layered
circuits of 14 and 16 qubits end with a pass that carries no gate and only
restores the standard order; the mixed and QFT circuits cover diagonal ops,
controls outside the tile and held-back phases under a permuted storage
order.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close, oracle_threads, rounded
from tests.gpu_helpers import state_from_host
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu


def _run(n, dtype, psi0, g, flags):
    h = state_from_host(n, dtype, psi0)
    try:
        sv.sv_run_circuit(h, g, flags)
        return sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)


def _passes(n, dtype, g, flags):
    return sv.sv_plan_inspect(n, dtype, g, flags)[1]


C128, C64 = sv.SV_C128, sv.SV_C64
# (kind, n, circuit, dtype): the planner keeps the relabelled plan for each
CASES = [
    ("layers", 14, lambda n: qc.layer_circuit(n, 100, n * 100 + 100), C128),
    ("layers", 14, lambda n: qc.layer_circuit(n, 100, n * 100 + 100), C64),
    ("layers", 16, lambda n: qc.layer_circuit(n, 100, n * 100 + 100), C128),
    ("layers", 17, lambda n: qc.layer_circuit(n, 40, n * 100 + 40), C64),
    ("layers", 18, lambda n: qc.layer_circuit(n, 40, n * 100 + 40), C128),
    ("layers", 19, lambda n: qc.layer_circuit(n, 20, n * 100 + 20), C64),
    ("mixed", 16, lambda n: mixed_circuit(n, 1500, 5 * n + 3), C64),
    ("mixed", 19, lambda n: mixed_circuit(n, 1500, 5 * n + 4), C128),
    ("qft+layers", 20, lambda n: np.concatenate([qc.qft_circuit(n), qc.layer_circuit(n, 20, 3)]), C128),
    ("qft+layers", 20, lambda n: np.concatenate([qc.qft_circuit(n), qc.layer_circuit(n, 20, 3)]), C64),
    # states past the last-level cache, many tiles per work-group
    ("layers", 25, lambda n: qc.layer_circuit(n, 12, n * 100 + 12), C128),
    ("layers", 26, lambda n: qc.layer_circuit(n, 12, n * 100 + 12), C64),
    ("mixed", 25, lambda n: mixed_circuit(n, 1000, 5 * n + 4), C128),
    ("mixed", 26, lambda n: mixed_circuit(n, 1500, 5 * n + 4), C64),
    ("qft+layers", 25, lambda n: np.concatenate([qc.qft_circuit(n), qc.layer_circuit(n, 10, 3)]), C128),
]


@pytest.mark.parametrize("kind,n,make,dtype", CASES,
                         ids=[f"{k}-{n}-{'c128' if d == C128 else 'c64'}" for k, n, _, d in CASES])
def test_relabelled_passes_match_oracle(kind, n, make, dtype):
    g = make(n)
    fixed = _passes(n, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)
    moved = _passes(n, dtype, g, sv.SV_FUSE)
    print(f"{kind} n={n} passes fixed {fixed} relabelled {moved}", flush=True)
    assert moved < fixed, "relabelling does not change this plan"
    psi0 = rounded(qc.random_state(n, 900 + n), dtype)
    ref = psi0.copy()
    with oracle_threads():
        oracle.run_circuit(ref, g)
    got = _run(n, dtype, psi0, g, sv.SV_FUSE)
    assert_close(got, ref, dtype, len(g), f"{kind} n={n} relabelled")
    base = _run(n, dtype, psi0, g, sv.SV_FUSE | sv.SV_NO_RELABEL)
    assert_close(base, ref, dtype, len(g), f"{kind} n={n} standard order")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_relabelled_qft_closed_form(dtype):
    """QFT after layers that leave qubits relabelled: the QFT part is checked
    against the closed form on the inverse of the layers."""
    n = 18
    layers = qc.layer_circuit(n, 30, 18)
    x = qc.random_basis_index(n, 5)
    g = np.concatenate([layers, qc.inverse_circuit(layers), qc.qft_circuit(n)])
    assert _passes(n, dtype, g, sv.SV_FUSE) < _passes(n, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_reset(h, x)
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)
    want = oracle.qft_basis_amplitudes(n, x, np.arange(1 << n))
    assert_close(got, want, dtype, len(g), "layers, inverse, QFT")


def test_no_relabel_rejected_without_fuse():
    h = sv.sv_create(6, sv.SV_C128)
    try:
        with pytest.raises(sv.SVError) as e:
            sv.sv_run_circuit(h, qc.layer_circuit(6, 2, 1), sv.SV_NO_RELABEL)
        assert e.value.status == sv.SV_EINVAL
        with pytest.raises(sv.SVError) as e:
            sv.sv_run_circuit(h, qc.layer_circuit(6, 2, 1), sv.SV_GRAPH | sv.SV_NO_RELABEL)
        assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(h)
