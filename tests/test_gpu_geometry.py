"""GPU: the tile geometry of a handle (sv_set_tile_geometry) and its tuner.

The tile pass (many gates per sweep of the state) runs with any geometry the
call accepts: fewer tile qubits, three register qubits, more or fewer fixed
low index bits. Each is checked against the oracle, with the generic and the
compiled kernels, and the tuner's choice is one of its candidates and gives
the same state."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from paper_1801_01037_amd import autotune
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close, rounded, state_from_host
from tests.test_plan import mixed_circuit

pytestmark = pytest.mark.gpu

GEOMETRIES = [(0, 0, -1), (10, 3, -1), (8, 4, 2), (12, 4, 5), (12, 4, 6), (6, 3, 0)]


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("geo", GEOMETRIES, ids=lambda g: "L%d_K%d_low%d" % g)
def test_geometries_match_the_oracle(dtype, geo):
    n = 14
    g = mixed_circuit(n, 250, 5 * n + sum(geo), mcu=True)
    psi0 = rounded(qc.random_state(n, 77), dtype)
    ref = psi0.copy()
    oracle.run_circuit(ref, g)
    for flags in (sv.SV_FUSE, sv.SV_FUSE | sv.SV_JIT, sv.SV_FUSE | sv.SV_NO_RELABEL):
        h = state_from_host(n, dtype, psi0)
        try:
            sv.sv_set_tile_geometry(h, *geo)
            sv.sv_run_circuit(h, g, flags)
            got = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        assert_close(got, ref, dtype, len(g), f"geometry {geo} flags {flags}")


def test_bad_geometries_are_rejected_and_leave_the_setting():
    n = 10
    g = qc.layer_circuit(n, 4, 3)
    h = sv.sv_create(n, sv.SV_C128)
    try:
        sv.sv_set_tile_geometry(h, 8, 3, 2)
        for bad in ((13, 0, -1), (3, 0, -1), (0, 2, -1), (0, 5, -1), (0, 0, 12), (0, 0, -2)):
            with pytest.raises(sv.SVError) as e:
                sv.sv_set_tile_geometry(h, *bad)
            assert e.value.status == sv.SV_EINVAL
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        ref = oracle.simulate(n, g)
        assert_close(sv.sv_copy_out(h), ref, sv.SV_C128, len(g), "after rejected geometries")
    finally:
        sv.sv_destroy(h)


def test_geometry_change_drops_the_captured_graph():
    """A replayed SV_GRAPH circuit is planned again after a geometry change."""
    n = 13
    g = qc.layer_circuit(n, 6, 4)
    ref = oracle.simulate(n, g)
    h = sv.sv_create(n, sv.SV_C128)
    try:
        for geo in ((0, 0, -1), (9, 3, 1), (9, 3, 1), (0, 0, -1)):
            sv.sv_set_tile_geometry(h, *geo)
            sv.sv_reset(h, 0)
            sv.sv_run_circuit(h, g, sv.SV_FUSE | sv.SV_GRAPH)
            assert_close(sv.sv_copy_out(h), ref, sv.SV_C128, len(g), f"graph after {geo}")
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_tuner_picks_a_candidate_and_the_same_state(dtype):
    n = 14
    g = qc.layer_circuit(n, 8, 6)
    cands = ((0, 0, -1), (10, 3, -1), (0, 0, 5))
    st = sv.StateVector(n, dtype)
    try:
        best, times = autotune.tune_tile_geometry(st, g, "test", candidates=cands, use_cache=False)
        assert best in cands
        assert set(times) == {"%d,%d,%d" % c for c in cands}
        assert all(t > 0 for t in times.values())
        st.reset(0)
        st.run(g, sv.SV_FUSE | sv.SV_JIT)
        assert_close(st.numpy().astype(np.complex128), oracle.simulate(n, g), dtype, len(g), "tuned")
    finally:
        st.close()
