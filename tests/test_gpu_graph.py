"""GPU: SV_GRAPH on sv_run_circuit. The first call captures the circuit's
launches in a HIP graph; later calls with the same gate list replay it. Every
replay must equal the run without SV_GRAPH bit for bit (and the oracle within
the stated bounds), with eager work and synchronizations between replays; a
different gate list or different flags capture again."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu

MODES = [0, sv.SV_FUSE, sv.SV_FUSE | sv.SV_NO_RELABEL, sv.SV_FUSE_DENSE]
MODE_IDS = ["per-gate", "fused", "fused-standard-order", "dense"]


def _with_toffoli(n, g):
    """The gate list with a doubly controlled gate in the middle, so planned
    segments alternate with a launch of its own."""
    mid = len(g) // 2
    t = qc.gate_mcu([0, n - 1], n // 2, qc.haar_su2(9, 1)[0])
    return np.concatenate([g[:mid], t, g[mid:]])


def _run(h, g, flags, x=0):
    sv.sv_reset(h, x)
    sv.sv_run_circuit(h, g, flags)
    return sv.sv_copy_out(h)


@pytest.mark.parametrize("flags", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_graph_replays_equal_the_direct_run(dtype, flags):
    n = 14
    g = _with_toffoli(n, qc.workload_layers_qft(n, 12, 5))
    h = sv.sv_create(n, dtype)
    try:
        direct = _run(h, g, flags, 3)
        outs = []
        for k in range(4):
            outs.append(_run(h, g, flags | sv.SV_GRAPH, 3))
            # eager work on the handle between replays
            sv.sv_apply_1q(h, k % n, qc.H_MATRIX)
            sv.sv_norm(h)
    finally:
        sv.sv_destroy(h)
    for k, o in enumerate(outs):
        assert np.array_equal(o, direct), f"replay {k}"
    assert_close(direct, oracle.simulate(n, g, 3), dtype, len(g), "graph")


def test_graph_recaptures_when_the_list_or_flags_change():
    n, dtype = 13, sv.SV_C128
    g1 = mixed_circuit(n, 200, 1)
    g2 = mixed_circuit(n, 200, 2)
    h = sv.sv_create(n, dtype)
    try:
        want1 = _run(h, g1, sv.SV_FUSE)
        want2 = _run(h, g2, sv.SV_FUSE)
        want1d = _run(h, g1, sv.SV_FUSE_DENSE)
        for g, f, w in ((g1, sv.SV_FUSE, want1), (g2, sv.SV_FUSE, want2), (g1, sv.SV_FUSE, want1),
                        (g1, sv.SV_FUSE_DENSE, want1d), (g1, sv.SV_FUSE, want1)):
            assert np.array_equal(_run(h, g, f | sv.SV_GRAPH), w)
        # the same list with one angle changed is a different list
        g3 = g1.copy()
        k = int(np.flatnonzero(g3["kind"] == qc.G_CPHASE)[0])
        g3[k]["m"][0] += 0.25
        assert np.array_equal(_run(h, g3, sv.SV_FUSE | sv.SV_GRAPH), _run(h, g3, sv.SV_FUSE))
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8])
def test_graph_on_small_registers(n):
    g = mixed_circuit(n, 60, 40 + n)
    for dtype in DTYPES:
        h = sv.sv_create(n, dtype)
        try:
            want = _run(h, g, sv.SV_FUSE)
            for _ in range(2):
                assert np.array_equal(_run(h, g, sv.SV_FUSE | sv.SV_GRAPH), want), (n, dtype)
            assert np.array_equal(_run(h, g, sv.SV_FUSE_DENSE | sv.SV_GRAPH),
                                  _run(h, g, sv.SV_FUSE_DENSE)), (n, dtype)
        finally:
            sv.sv_destroy(h)


def test_graph_at_a_streaming_size():
    """25 qubits complex128 (tile passes with the nontemporal hint)."""
    n = 25
    g = qc.layer_circuit(n, 6, 8)
    a = sv.StateVector(n, sv.SV_C128)
    b = sv.StateVector(n, sv.SV_C128)
    try:
        a.run(g, sv.SV_FUSE)
        for _ in range(2):
            b.reset(0)
            b.run(g, sv.SV_FUSE | sv.SV_GRAPH)
        c = sv.sv_compare(a.handle, b.handle)
    finally:
        a.close()
        b.close()
    assert c["max_abs"] == 0.0


def test_graph_replays_are_profiled_as_one_launch():
    n = 12
    g = qc.layer_circuit(n, 10, 3)
    h = sv.sv_create(n, sv.SV_C64)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE | sv.SV_GRAPH)   # capture
        sv.sv_profile(h, True)
        for _ in range(3):
            sv.sv_run_circuit(h, g, sv.SV_FUSE | sv.SV_GRAPH)
        sv.sv_profile(h, False)
        prof = sv.sv_profile_read(h)
    finally:
        sv.sv_destroy(h)
    assert set(prof) == {"graph"}
    assert prof["graph"]["launches"] == 3
    assert prof["graph"]["bytes"] > 0
