"""GPU: many circuits run as one batch (sv_batch_run, level launches) give the
same result as each circuit run alone, and match the oracle."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close

pytestmark = pytest.mark.gpu


def _specs(count, seed, n_lo=10, n_hi=18, d_lo=4, d_hi=30):
    return qc.batch_specs(seed, count, n_lo, n_hi, d_lo, d_hi)


def _run_alone(n, dtype, g):
    """The circuit run alone with SV_FUSE, which makes the plan a batch uses,
    so results are bitwise equal."""
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_run_circuit(h, g, sv.SV_FUSE)
        return sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)


def test_batch_of_full_tiles():
    """Every circuit fills a whole tile (complex128, n >= 12): all threads of
    each work-group hold amplitudes."""
    dtype = sv.SV_C128
    specs = _specs(6, 41, 12, 16, 4, 12)
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_run(b, plans)
        sv.sv_batch_times(b, len(plans))
        outs = [sv.sv_copy_out(h) for h in states]
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    for (n, d, s), g, got in zip(specs, circuits, outs):
        assert np.array_equal(got, _run_alone(n, dtype, g)), (n, d)


def test_small_circuits_finish_before_a_large_one():
    """Levels take the circuits with the least remaining work first: sixteen
    10-qubit circuits end before one 22-qubit circuit of the same batch, and
    every result equals the circuit run alone."""
    dtype = sv.SV_C64
    specs = [(22, 30, 901)] + [(10, 12, 910 + i) for i in range(16)]
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_run(b, plans)
        start, end = sv.sv_batch_times(b, len(plans))
        outs = [sv.sv_copy_out(h) for h in states]
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    assert max(end[1:]) < end[0], (end[0], max(end[1:]))
    for (n, d, s), g, got in zip(specs, circuits, outs):
        assert np.array_equal(got, _run_alone(n, dtype, g)), (n, d)


@pytest.mark.parametrize("flags", [0, sv.SV_GRAPH], ids=["launches", "graph"])
@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_batch_equals_alone_and_oracle(dtype, flags):
    specs = _specs(24, 5)
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_run(b, plans, flags=flags)
        start, end = sv.sv_batch_times(b, len(plans))
        outs = [sv.sv_copy_out(h) for h in states]
        if flags:                                   # replay the captured graph
            for h in states:
                sv.sv_reset(h, 0)
                sv.sv_synchronize(h)
            sv.sv_batch_run(b, plans, flags=flags)
            sv.sv_batch_times(b, len(plans))
            again = [sv.sv_copy_out(h) for h in states]
            assert all(np.array_equal(x, y) for x, y in zip(outs, again))
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    assert np.all(end >= start) and np.all(start >= 0)
    for (n, d, s), g, got in zip(specs, circuits, outs):
        alone = _run_alone(n, dtype, g)
        assert np.array_equal(got, alone), (n, d)          # same alone and in the mix
        if n <= 16:
            assert_close(got, oracle.simulate(n, g), dtype, len(g), f"batch n={n} d={d}")


def test_batch_in_pass_ranges_and_configs():
    """Running plans in two chunks of passes, under different launch
    configurations, gives the same bits as one full run."""
    dtype = sv.SV_C64
    specs = _specs(12, 9, 12, 20, 10, 40)
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    ref = [_run_alone(n, dtype, g) for (n, _, _), g in zip(specs, circuits)]
    for bpc, tpt in [(1, 1), (2, 8), (4, 64)]:
        states = [sv.sv_create(n, dtype) for n, _, _ in specs]
        plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
        b = sv.sv_batch_create(dtype)
        try:
            sv.sv_batch_config(b, bpc, tpt)
            npass = np.array([sv.sv_plan_passes(p) for p in plans], dtype=np.int32)
            half = npass // 2
            sv.sv_batch_run(b, plans, np.zeros_like(half), half)
            sv.sv_batch_run(b, plans, half, npass - half)
            outs = [sv.sv_copy_out(h) for h in states]
        finally:
            sv.sv_batch_destroy(b)
            for p in plans:
                sv.sv_plan_destroy(p)
            for h in states:
                sv.sv_destroy(h)
        for r, got in zip(ref, outs):
            assert np.array_equal(r, got), (bpc, tpt)


def test_run_plan_matches_fused_run():
    n, dtype = 17, sv.SV_C128
    g = qc.workload_layers_qft(n, 12, 3)
    h = sv.sv_create(n, dtype)
    try:
        p = sv.sv_plan_create(h, g)
        k = sv.sv_plan_passes(p)
        sv.sv_run_plan(p, 0, k // 2)
        sv.sv_run_plan(p, k // 2, k - k // 2)
        got = sv.sv_copy_out(h)
        sv.sv_plan_destroy(p)
    finally:
        sv.sv_destroy(h)
    assert np.array_equal(got, _run_alone(n, dtype, g))


def test_graph_recaptured_after_a_plan_is_replaced():
    """A captured batch graph belongs to the plans it was captured for: after a
    plan is destroyed and another one made (often at the same host address),
    the next SV_GRAPH run captures again and runs the new plan's passes."""
    dtype = sv.SV_C64
    specs = _specs(4, 77, 12, 14, 4, 10)
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    first = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    second = [qc.layer_circuit(n, d + 3, s + 1) for n, d, s in specs]
    b = sv.sv_batch_create(dtype)
    plans = []
    try:
        plans = [sv.sv_plan_create(h, g) for h, g in zip(states, first)]
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)
        outs1 = [sv.sv_copy_out(h) for h in states]
        for p in plans:
            sv.sv_plan_destroy(p)
        plans = []
        for h in states:
            sv.sv_reset(h, 0)
            sv.sv_synchronize(h)
        plans = [sv.sv_plan_create(h, g) for h, g in zip(states, second)]
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)
        outs2 = [sv.sv_copy_out(h) for h in states]
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    for (n, _, _), g1, g2, o1, o2 in zip(specs, first, second, outs1, outs2):
        assert np.array_equal(o1, _run_alone(n, dtype, g1))
        assert np.array_equal(o2, _run_alone(n, dtype, g2))


def test_batch_rejects_bad_requests():
    h1 = sv.sv_create(10, sv.SV_C64)
    h2 = sv.sv_create(10, sv.SV_C128)
    g = qc.layer_circuit(10, 2, 1)
    p1, p2 = sv.sv_plan_create(h1, g), sv.sv_plan_create(h2, g)
    b = sv.sv_batch_create(sv.SV_C64)
    try:
        with pytest.raises(sv.SVError):
            sv.sv_batch_run(b, [p1, p2])               # mixed dtypes
        with pytest.raises(sv.SVError):
            sv.sv_batch_run(b, [p1, p1])               # one state twice
        with pytest.raises(sv.SVError):
            sv.sv_batch_run(b, [p1], [0], [10 ** 6])   # pass range outside the plan
        with pytest.raises(sv.SVError):
            sv.sv_batch_config(b, 0, 8)
    finally:
        sv.sv_batch_destroy(b)
        sv.sv_plan_destroy(p1)
        sv.sv_plan_destroy(p2)
        sv.sv_destroy(h1)
        sv.sv_destroy(h2)


@pytest.mark.skip(reason="the persistent work-queue batch kernel this exercised is switched off: "
                         "it hung on the GPU twice (relaxed, then acquire polls of the "
                         "per-circuit counters); batches now run one launch per pass level "
                         "with no waits, and sv_batch_set_wait_limit is gone with it")
def test_expired_waits_are_reported_and_the_launch_ends():
    """A zero wait bound makes every dependent task give up (forced from the
    host); the launch still ends and the run reports SV_EDEVICE."""
    dtype = sv.SV_C64
    n = 16
    g = qc.layer_circuit(n, 30, 2)
    h = sv.sv_create(n, dtype)
    p = sv.sv_plan_create(h, g)
    b = sv.sv_batch_create(dtype)
    try:
        assert sv.sv_plan_passes(p) > 1
        sv.sv_batch_set_wait_limit(b, 0.0)
        sv.sv_batch_run(b, [p])
        with pytest.raises(sv.SVError) as ei:
            sv.sv_batch_times(b, 1)
        assert ei.value.status == sv.SV_EDEVICE
        sv.sv_batch_set_wait_limit(b, 10000.0)     # a normal run afterwards is fine
        sv.sv_reset(h, 0)
        sv.sv_synchronize(h)
        sv.sv_batch_run(b, [p])
        sv.sv_batch_times(b, 1)
        got = sv.sv_copy_out(h)
    finally:
        sv.sv_batch_destroy(b)
        sv.sv_plan_destroy(p)
        sv.sv_destroy(h)
    assert np.array_equal(got, _run_alone(n, dtype, g))


# ---- the persistent launch for small circuits ---------------------------------

@pytest.mark.parametrize("max_tiles", [1, 16, 1 << 20], ids=["one-tile", "up-to-16", "all"])
@pytest.mark.parametrize("flags", [0, sv.SV_GRAPH], ids=["launches", "graph"])
@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_persistent_batch_equals_alone(dtype, flags, max_tiles):
    """Circuits small enough run whole in one persistent launch on the batch's
    second stream (work-group w takes circuits w, w + G, ...), the rest in level
    launches beside it; every result equals the circuit run alone, bit for bit,
    also on a graph replay, and every circuit's clock interval is filled."""
    specs = _specs(20, 21, 4, 17, 5, 60)
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_persist(b, max_tiles)
        sv.sv_batch_run(b, plans, flags=flags)
        start, end = sv.sv_batch_times(b, len(plans))
        outs = [sv.sv_copy_out(h) for h in states]
        if flags:
            for h in states:
                sv.sv_reset(h, 0)
                sv.sv_synchronize(h)
            sv.sv_batch_run(b, plans, flags=flags)
            sv.sv_batch_times(b, len(plans))
            again = [sv.sv_copy_out(h) for h in states]
            assert all(np.array_equal(x, y) for x, y in zip(outs, again))
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    assert np.all(end > start) and np.all(start >= 0)
    for (n, d, s), g, got in zip(specs, circuits, outs):
        assert np.array_equal(got, _run_alone(n, dtype, g)), (n, d)
        if n <= 12:
            assert_close(got, oracle.simulate(n, g), dtype, len(g), f"persistent n={n} d={d}")


def test_persistent_small_circuits_finish_first():
    """With the persistent launch (on the batch's second stream, beside the
    levels), the small circuits of a batch all end before the large one."""
    dtype = sv.SV_C64
    specs = [(22, 20, 31)] + [(10, 30, 40 + i) for i in range(32)]
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_persist(b, 1)
        sv.sv_batch_run(b, plans)
        start, end = sv.sv_batch_times(b, len(plans))
        outs = [sv.sv_copy_out(h) for h in states]
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
    assert max(end[1:]) < end[0], (end[0], max(end[1:]))
    for (n, d, s), g, got in zip(specs[1:], circuits[1:], outs[1:]):
        assert np.array_equal(got, _run_alone(n, dtype, g))


def test_persist_rejects_bad_values():
    b = sv.sv_batch_create(sv.SV_C64)
    try:
        for v in (-1, (1 << 20) + 1):
            with pytest.raises(sv.SVError) as e:
                sv.sv_batch_persist(b, v)
            assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_batch_destroy(b)


@pytest.mark.parametrize("flags", [sv.SV_FUSE, sv.SV_FUSE | sv.SV_GRAPH], ids=["direct", "graph"])
def test_run_batch_one_call_mixed_states(flags):
    """sv_run_batch: complex64 and complex128 states of several sizes and
    streams, a circuit with a Toffoli (batched), one on 3 qubits (run alone),
    an empty circuit, a 24-qubit circuit (pass by pass on the batch's third
    stream); every result equals the circuit run alone with SV_FUSE."""
    import torch
    side = torch.cuda.Stream()
    cases = [(12, sv.SV_C128, qc.layer_circuit(12, 6, 71), None),
             (14, sv.SV_C64, qc.layer_circuit(14, 8, 72), side.cuda_stream),
             (10, sv.SV_C64, np.concatenate([qc.layer_circuit(10, 3, 73),
                                             qc.gate_mcu((0, 4), 9, qc.X_MATRIX),
                                             qc.layer_circuit(10, 2, 74)]), None),
             (3, sv.SV_C128, qc.layer_circuit(3, 5, 75), None),
             (9, sv.SV_C128, qc.layer_circuit(9, 0, 76), None),
             (16, sv.SV_C128, qc.qft_circuit(16), side.cuda_stream),
             (11, sv.SV_C64, qc.qft_circuit(11), None),
             (24, sv.SV_C64, qc.layer_circuit(24, 2, 77), None)]
    states = [sv.sv_create(n, dt, st) for n, dt, _, st in cases]
    try:
        for h, (n, _, _, _) in zip(states, cases):
            sv.sv_reset(h, qc.random_basis_index(n, 700 + n))
        sv.sv_run_batch(states, [g for _, _, g, _ in cases], flags)
        outs = [sv.sv_copy_out(h) for h in states]
    finally:
        for h in states:
            sv.sv_destroy(h)
    for (n, dt, g, _), got in zip(cases, outs):
        h = sv.sv_create(n, dt)
        try:
            sv.sv_reset(h, qc.random_basis_index(n, 700 + n))
            sv.sv_run_circuit(h, g, sv.SV_FUSE)
            want = sv.sv_copy_out(h)
        finally:
            sv.sv_destroy(h)
        assert np.array_equal(got, want), (n, dt, len(g))
        ref = oracle.basis_state(n, qc.random_basis_index(n, 700 + n))
        oracle.run_circuit(ref, g)
        assert_close(got, ref, dt, max(len(g), 1), f"n={n}")


def test_run_batch_rejects_before_running():
    """A repeated state or an invalid gate in any circuit is reported before
    any work is queued: every state keeps its value."""
    a = sv.sv_create(10, sv.SV_C128)
    b = sv.sv_create(12, sv.SV_C128)
    try:
        sv.sv_reset(a, 5)
        sv.sv_reset(b, 6)
        good = qc.layer_circuit(10, 4, 81)
        bad = qc.layer_circuit(12, 4, 82)
        bad[3]["target"] = 12                      # outside the 12-qubit register
        with pytest.raises(sv.SVError) as e:
            sv.sv_run_batch([a, b], [good, bad])
        assert e.value.status == sv.SV_EINVAL
        with pytest.raises(sv.SVError) as e:
            sv.sv_run_batch([a, a], [good, good])
        assert e.value.status == sv.SV_EINVAL
        assert np.array_equal(sv.sv_copy_out(a), oracle.basis_state(10, 5))
        assert np.array_equal(sv.sv_copy_out(b), oracle.basis_state(12, 6))
    finally:
        sv.sv_destroy(a)
        sv.sv_destroy(b)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("flags", [0, sv.SV_GRAPH], ids=["direct", "graph"])
def test_large_circuits_on_a_third_stream(dtype, flags):
    """sv_batch_solo: circuits of at least 4 tiles per pass (n >= 14) run pass
    by pass on a third stream while 2-tile circuits take the levels and 1-tile
    ones the persistent launch. Two runs in a row (the second a graph replay
    under SV_GRAPH); every result equals the circuit run alone, and every
    circuit has clocks."""
    specs = [(14, 20, 1301), (16, 8, 1302), (15, 12, 1303), (10, 30, 1304),
             (12, 10, 1305), (13, 16, 1306), (13, 6, 1307), (14, 0, 1308)]
    circuits = [qc.layer_circuit(n, d, s) for n, d, s in specs]
    states = [sv.sv_create(n, dtype) for n, _, _ in specs]
    plans = [sv.sv_plan_create(h, g) for h, g in zip(states, circuits)]
    b = sv.sv_batch_create(dtype)
    try:
        sv.sv_batch_persist(b, 1)
        sv.sv_batch_solo(b, 4)
        for _ in range(2):
            for h, (n, _, s) in zip(states, specs):
                sv.sv_reset(h, qc.random_basis_index(n, s))
            sv.sv_batch_run(b, plans, flags=flags)
            start, end = sv.sv_batch_times(b, len(plans))
            outs = [sv.sv_copy_out(h) for h in states]
            for (n, d, s), g, got, t0, t1 in zip(specs, circuits, outs, start, end):
                h = sv.sv_create(n, dtype)
                try:
                    sv.sv_reset(h, qc.random_basis_index(n, s))
                    sv.sv_run_circuit(h, g, sv.SV_FUSE)
                    want = sv.sv_copy_out(h)
                finally:
                    sv.sv_destroy(h)
                assert np.array_equal(got, want), (n, d)
                assert 0.0 <= t0 <= t1, (n, d, t0, t1)
                if d:
                    assert t1 > 0.0, (n, d)
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for h in states:
            sv.sv_destroy(h)
