"""The SV_FUSE planner on the host: every gate is applied exactly once, and any
two gates that share a qubit keep their order unless both are diagonal
(diagonal gates commute with each other). Runs without a GPU."""
import math

import numpy as np
import pytest

import paper_1801_01037_amd as sv
import qcircuits as qc


def _is_diag(g):
    if int(g["kind"]) == qc.G_CPHASE:
        return True
    m = g["m"]
    if not (m[0] == 1 and m[1] == 0 and m[2] == 0 and m[3] == 0 and m[4] == 0 and m[5] == 0):
        return False
    return abs(m[6] ** 2 + m[7] ** 2 - 1.0) <= 4e-16


def _qubits(g):
    if int(g["kind"]) == qc.G_MCU:
        m = qc.gate_control_mask(g)
        return {int(g["target"])} | {q for q in range(64) if (m >> q) & 1}
    return {int(g["target"])} | ({int(g["control"])} if int(g["control"]) >= 0 else set())


def check_plan_order(n, dtype, gates, strict=False):
    """strict: every non-diagonal gate has an op of its own (no 4x4 fusion)."""
    gate_op, passes, groups, ops = sv.sv_plan_inspect(n, dtype, gates)
    assert (gate_op >= 0).all() and (gate_op < ops).all()
    diag = np.array([_is_diag(g) for g in gates])
    by_qubit = {}
    for i, g in enumerate(gates):
        for q in _qubits(g):
            by_qubit.setdefault(q, []).append(i)
    for q, idx in by_qubit.items():
        for a in range(len(idx)):
            for b in range(a + 1, len(idx)):
                i, j = idx[a], idx[b]
                if diag[i] and diag[j]:
                    continue
                # gates merged into one op are applied as one product, in order
                if strict:
                    assert gate_op[i] < gate_op[j], (q, i, j, gate_op[i], gate_op[j])
                else:
                    assert gate_op[i] <= gate_op[j], (q, i, j, gate_op[i], gate_op[j])
    if strict:
        nondiag_ops = gate_op[~diag]
        assert len(set(nondiag_ops.tolist())) == len(nondiag_ops)   # one op per such gate
    return passes, groups, ops


@pytest.fixture
def no_fusion(monkeypatch):
    monkeypatch.setenv("SV_TILE_FUSE4", "0")


def mixed_circuit(n, count, seed, mcu=False):
    """Random gates of every kind a pass holds: 2x2, controlled 2x2, CNOT,
    controlled phase, one-qubit phase, X; with `mcu` (n >= 3) also gates with
    two to four controls (Toffoli among them)."""
    rng = np.random.default_rng(seed)
    su2 = qc.haar_su2(seed, count)
    out = []
    kinds = 8 if (mcu and n >= 3) else 6
    for i in range(count):
        kind = int(rng.integers(0, kinds)) if n > 1 else 0
        if kind >= 6:
            t = int(rng.integers(0, n))
            k = int(rng.integers(2, min(4, n - 1) + 1))
            ctrls = rng.choice([q for q in range(n) if q != t], size=k, replace=False)
            out.append(qc.gate_mcu(ctrls, t, qc.X_MATRIX if kind == 6 else su2[i]))
            continue
        t = int(rng.integers(0, n))
        c = int(rng.integers(0, n - 1)) if n > 1 else 0
        c = c + 1 if c >= t else c
        if kind == 0:
            out.append(qc.gate_u(t, su2[i]))
        elif kind == 1:
            out.append(qc.gate_cu(c, t, su2[i]))
        elif kind == 2:
            out.append(qc.gate_cnot(c, t))
        elif kind == 3:
            out.append(qc.gate_cphase(c, t, float(rng.uniform(-7, 7))))
        elif kind == 4:
            ph = float(rng.uniform(-3, 3))
            out.append(qc.gate_u(t, (1, 0, 0, 0, 0, 0, math.cos(ph), math.sin(ph))))
        else:
            out.append(qc.gate_u(t, qc.X_MATRIX))
    return np.concatenate(out)


@pytest.mark.parametrize("dtype", [sv.SV_C128, sv.SV_C64], ids=["c128", "c64"])
def test_workload_plans_are_legal(dtype):
    shapes = {}
    for name, n, g in [("qft30", 30, qc.qft_circuit(30)),
                       ("layers30", 30, qc.layer_circuit(30, 20, 1)),
                       ("layers_qft16", 16, qc.workload_layers_qft(16, 100, 0)),
                       ("layers34", 34, qc.layer_circuit(34, 10, 1))]:
        shapes[name] = check_plan_order(n, dtype, g)
    assert shapes["qft30"][0] <= 6          # QFT(30) needs only a few sweeps
    assert shapes["layers30"][0] <= 40


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 13, 17, 22, 26, 28])
def test_mixed_circuit_plans_are_legal(n):
    """Every gate is applied once and in an order that keeps every pair of
    gates on a common qubit (26 qubits and up: groups chosen by coverage)."""
    for seed in range(3):
        g = mixed_circuit(n, 300, seed + 100 * n)
        for dtype in (sv.SV_C128, sv.SV_C64):
            check_plan_order(n, dtype, g)


@pytest.mark.parametrize("n", [5, 13, 22])
def test_unfused_plans_keep_every_order(n, no_fusion):
    for seed in range(2):
        g = mixed_circuit(n, 300, seed + 7 * n)
        check_plan_order(n, sv.SV_C128, g, strict=True)
    check_plan_order(30, sv.SV_C128, qc.layer_circuit(30, 20, 1), strict=True)


def test_fusion_reduces_ops():
    g = qc.layer_circuit(30, 20, 1)
    _, passes, groups, fused_ops = sv.sv_plan_inspect(30, sv.SV_C128, g)
    assert fused_ops < 0.62 * len(g)
    assert groups * 8 < len(g)          # light-cone groups fill the register qubits


def test_plan_rejects_bad_gates():
    with pytest.raises(sv.SVError):
        sv.sv_plan_inspect(4, sv.SV_C128, qc.gate_cnot(2, 2))
    with pytest.raises(sv.SVError):
        sv.sv_plan_inspect(4, sv.SV_C128, qc.gate_u(4, qc.X_MATRIX))


@pytest.mark.parametrize("n", [3, 4, 9, 13, 22])
def test_plans_hold_gates_with_several_controls(n):
    """Toffoli and other several-control gates join tile passes: every gate is
    placed once and gates sharing a qubit keep their order, in both storage
    orders."""
    for seed in range(3):
        g = mixed_circuit(n, 300, seed + 31 * n, mcu=True)
        assert (g["kind"] == qc.G_MCU).sum() > 10
        for dtype in (sv.SV_C128, sv.SV_C64):
            check_plan_order(n, dtype, g)
            sv.sv_plan_inspect(n, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)


def test_several_control_plans_keep_every_order(no_fusion):
    g = mixed_circuit(14, 400, 5, mcu=True)
    check_plan_order(14, sv.SV_C128, g, strict=True)


def test_malformed_control_masks_are_rejected():
    # the target among the controls, a control at or above n, no control at all
    for bad in (qc.gate_mcu((0, 2), 2, qc.X_MATRIX), qc.gate_mcu((0, 6), 2, qc.X_MATRIX),
                qc.gate_mcu((), 2, qc.X_MATRIX)):
        with pytest.raises(sv.SVError) as e:
            sv.sv_plan_inspect(6, sv.SV_C128, bad)
        assert e.value.status == sv.SV_EINVAL


def test_dense_plans_take_gates_of_up_to_five_qubits():
    four = qc.gate_mcu((0, 3, 5, 7), 9, qc.X_MATRIX)    # five qubits: one block
    five = qc.gate_mcu((0, 3, 5, 7, 8), 9, qc.X_MATRIX)  # six: too wide
    masks, mats = sv.sv_plan_dense_inspect(12, four)
    assert len(masks) == 1 and int(masks[0]) == 0b1010101001
    # the block is the four-control X: an exchange of the two columns whose
    # four control bits are set, identity elsewhere
    assert np.allclose(np.abs(mats[0]) ** 2 @ np.ones(32), 1.0)
    with pytest.raises(sv.SVError) as e:
        sv.sv_plan_dense_inspect(12, five, cap=4)
    assert e.value.status == sv.SV_EUNSUPPORTED


# ---- relabelling between passes (non-sequential storage) ---------------------

@pytest.mark.parametrize("dtype", [sv.SV_C128, sv.SV_C64], ids=["c128", "c64"])
def test_relabelling_cuts_passes_of_layered_circuits(dtype):
    """Every tile must hold the index bits of one 128-byte line; relabelling
    puts the next gates' qubits there instead of qubits 0..2 (0..3 for
    complex64), so a layered circuit needs far fewer passes."""
    g = qc.layer_circuit(30, 20, 1)
    fixed = sv.sv_plan_inspect(30, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)[1]
    moved = sv.sv_plan_inspect(30, dtype, g, sv.SV_FUSE)[1]
    assert fixed >= 25 and moved <= 18, (fixed, moved)
    g = qc.layer_circuit(18, 40, 1840)
    fixed = sv.sv_plan_inspect(18, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)[1]
    moved = sv.sv_plan_inspect(18, dtype, g, sv.SV_FUSE)[1]
    assert moved * 2 < fixed, (fixed, moved)


def test_relabelling_never_adds_passes_and_keeps_order():
    """Passes that restore the standard order are counted; the planner keeps
    the fixed-order plan when relabelling would not save a pass. Gate order
    per qubit holds in either plan."""
    rng = np.random.default_rng(77)
    for trial in range(60):
        n = int(rng.integers(1, 35))
        kind = trial % 3
        if kind == 0:
            g = qc.layer_circuit(n, int(rng.integers(1, 40)), trial)
        elif kind == 1:
            g = qc.qft_circuit(n)
        else:
            g = np.concatenate([qc.qft_circuit(n), qc.layer_circuit(n, 5, trial)])
        for dtype in (sv.SV_C128, sv.SV_C64):
            fixed = sv.sv_plan_inspect(n, dtype, g, sv.SV_FUSE | sv.SV_NO_RELABEL)[1]
            moved = sv.sv_plan_inspect(n, dtype, g, sv.SV_FUSE)[1]
            assert moved <= fixed, (n, kind, fixed, moved)
            if n <= 20 and trial % 6 == 0:
                check_plan_order(n, dtype, g)


def test_no_relabel_needs_fuse():
    g = qc.layer_circuit(5, 2, 1)
    with pytest.raises(sv.SVError) as e:
        sv.sv_plan_inspect(5, sv.SV_C128, g, sv.SV_FUSE_DENSE | sv.SV_NO_RELABEL)
    assert e.value.status == sv.SV_EUNSUPPORTED


@pytest.mark.parametrize("dtype,shape", [
    (sv.SV_C128, {"qft": (3, 9, 59), "layers": (16, 72, 361)}),
    (sv.SV_C64, {"qft": (4, 9, 59), "layers": (17, 68, 345)}),
], ids=["c128", "c64"])
def test_benchmark_plans_do_not_grow(dtype, shape):
    """The plans of the 30-qubit benchmark step (QFT, depth-20 layers) keep
    at most the passes, register groups and ops they have now: a planner
    change that makes them longer shows here before it shows in the timings.
    (Complex64 takes the plans with six fixed low bits: as many or fewer
    passes, runs of 512 B; the QFT has one group more than with four.)"""
    for name, g in (("qft", qc.qft_circuit(30)), ("layers", qc.layer_circuit(30, 20, 1))):
        _, passes, groups, ops = sv.sv_plan_inspect(30, dtype, g, sv.SV_FUSE)
        p0, g0, o0 = shape[name]
        assert passes <= p0 and groups <= g0 and ops <= o0, (name, passes, groups, ops)


# ---- passes compiled at run time (SV_JIT) ------------------------------------

def test_pass_programs_compile_on_the_host():
    """The programs SV_FUSE | SV_JIT writes for a plan compile with hipRTC
    without a device: layered passes (one program per distinct pass shape),
    several-control gates, diagonal ops (the QFT), both storage orders, both
    precisions."""
    g = np.concatenate([qc.layer_circuit(14, 6, 3), mixed_circuit(14, 60, 4, mcu=True)])
    for dtype in (sv.SV_C128, sv.SV_C64):
        k = sv.sv_plan_jit_check(14, dtype, g)
        assert 1 <= k <= sv.sv_plan_inspect(14, dtype, g)[1]
        assert sv.sv_plan_jit_check(14, dtype, g, sv.SV_FUSE | sv.SV_JIT | sv.SV_NO_RELABEL) >= 1
    assert sv.sv_plan_jit_check(12, sv.SV_C128, qc.qft_circuit(12)) >= 1
    assert sv.sv_plan_jit_check(16, sv.SV_C64, qc.workload_layers_qft(16, 4, 1)) >= 1
    with pytest.raises(sv.SVError) as e:
        sv.sv_plan_jit_check(6, sv.SV_C128, g[:4], sv.SV_FUSE)
    assert e.value.status == sv.SV_EINVAL
