"""GPU: tile passes compiled at run time for their own program (SV_JIT).

A compiled pass applies the same device functions as the generic tile kernel
(with the op kinds and register positions fixed in the code), so its results
must equal the generic kernel's bit for bit, and the oracle within the stated
bounds: mixed circuits with every op kind (controls in registers, on other
tile bits and outside the tile; several controls; exchanges folded into
write-backs), both storage orders, small registers, streaming sizes, and under
SV_GRAPH."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, STREAMING, STREAMING_IDS, assert_close
from tests.gpu_helpers import oracle_threads, rounded, state_from_host
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu

JIT = sv.SV_FUSE | sv.SV_JIT


def _run(n, dtype, psi0, g, flags, x=None):
    h = state_from_host(n, dtype, psi0) if psi0 is not None else sv.sv_create(n, dtype)
    try:
        if x is not None:
            sv.sv_reset(h, x)
        sv.sv_run_circuit(h, g, flags)
        return sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [2, 5, 12, 16, 20])
def test_compiled_passes_equal_the_generic_kernel(dtype, n):
    g = mixed_circuit(n, 300, 19 * n + 1, mcu=n >= 3)
    psi0 = rounded(qc.random_state(n, 410 + n), dtype)
    want = _run(n, dtype, psi0, g, sv.SV_FUSE)
    for flags in (JIT, JIT | sv.SV_NO_RELABEL):
        got = _run(n, dtype, psi0, g, flags)
        if flags & sv.SV_NO_RELABEL:
            assert np.array_equal(got, _run(n, dtype, psi0, g, sv.SV_FUSE | sv.SV_NO_RELABEL))
        else:
            assert np.array_equal(got, want), f"n={n} flags={flags}"
    ref = psi0.copy()
    oracle.run_circuit(ref, g)
    assert_close(want, ref, dtype, len(g), f"jit n={n}")


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_layers_and_qft_compiled(dtype):
    """Layered passes are compiled; QFT passes (diagonal ops) keep the
    generic kernel; together against the oracle."""
    n = 18
    g = qc.workload_layers_qft(n, 30, 2)
    got = _run(n, dtype, None, g, JIT, 5)
    assert np.array_equal(got, _run(n, dtype, None, g, sv.SV_FUSE, 5))
    assert_close(got, oracle.simulate(n, g, 5), dtype, len(g), "layers+qft")


@pytest.mark.parametrize("n,dtype", STREAMING, ids=STREAMING_IDS)
def test_compiled_passes_at_streaming_sizes(n, dtype):
    g = np.concatenate([qc.layer_circuit(n, 8, n + 5), mixed_circuit(n, 200, n, mcu=True)])
    psi0 = rounded(qc.random_state(n, 420 + n), dtype)
    got = _run(n, dtype, psi0, g, JIT)
    ref = psi0.copy()
    with oracle_threads():
        oracle.run_circuit(ref, g)
    assert_close(got, ref, dtype, len(g), f"jit n={n}")
    assert np.array_equal(got, _run(n, dtype, psi0, g, sv.SV_FUSE))


def test_compiled_passes_under_graph_replay():
    n, dtype = 15, sv.SV_C128
    g = qc.layer_circuit(n, 16, 9)
    want = _run(n, dtype, None, g, sv.SV_FUSE)
    h = sv.sv_create(n, dtype)
    try:
        for _ in range(3):
            sv.sv_reset(h, 0)
            sv.sv_run_circuit(h, g, JIT | sv.SV_GRAPH)
            assert np.array_equal(sv.sv_copy_out(h), want)
            sv.sv_apply_1q(h, 3, qc.H_MATRIX)   # eager work between replays
    finally:
        sv.sv_destroy(h)


def test_jit_needs_fuse():
    h = sv.sv_create(6, sv.SV_C128)
    try:
        for flags in (sv.SV_JIT, sv.SV_JIT | sv.SV_FUSE_DENSE):
            with pytest.raises(sv.SVError) as e:
                sv.sv_run_circuit(h, qc.layer_circuit(6, 2, 1), flags)
            assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(h)
