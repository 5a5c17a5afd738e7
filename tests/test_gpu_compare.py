"""GPU: sv_compare, the FP64 comparison of two states on the device (the error
statement of a complex64 result against complex128), against numpy on the
same rounded amplitudes."""
import numpy as np
import pytest

import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import rounded, state_from_host

pytestmark = pytest.mark.gpu

C128, C64 = sv.SV_C128, sv.SV_C64
PAIRS = [(C64, C128), (C128, C64), (C128, C128), (C64, C64)]
PAIR_IDS = ["c64-c128", "c128-c64", "c128-c128", "c64-c64"]


def _numpy_figures(a, b):
    d = a.astype(np.complex128) - b.astype(np.complex128)
    return {"max_abs": float(np.max(np.abs(d))), "sq_err": float(np.sum(np.abs(d) ** 2)),
            "norm_a": float(np.sum(np.abs(a.astype(np.complex128)) ** 2)),
            "norm_b": float(np.sum(np.abs(b.astype(np.complex128)) ** 2))}


@pytest.mark.parametrize("da,db", PAIRS, ids=PAIR_IDS)
@pytest.mark.parametrize("n", [1, 3, 12, 21, 25])
def test_compare_matches_numpy(da, db, n):
    psi = qc.random_state(n, 500 + n)
    # b: psi; a: psi with a seeded perturbation, one amplitude pushed further
    noise = qc.random_state(n, 600 + n) * 1e-6
    pert = psi + noise
    pert[(1 << n) // 3] += 0.01
    a_host, b_host = rounded(pert, da), rounded(psi, db)
    ha = state_from_host(n, da, a_host)
    hb = state_from_host(n, db, b_host)
    try:
        got = sv.sv_compare(ha, hb)
        again = sv.sv_compare(ha, hb)
    finally:
        sv.sv_destroy(ha)
        sv.sv_destroy(hb)
    want = _numpy_figures(a_host, b_host)
    assert got["max_abs"] == pytest.approx(want["max_abs"], rel=1e-14, abs=0)
    for k in ("sq_err", "norm_a", "norm_b"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=0), k
    assert got["rel_l2"] == pytest.approx((want["sq_err"] / want["norm_b"]) ** 0.5, rel=1e-12)
    assert got == again   # a fixed reduction tree: the same bits on every call


@pytest.mark.parametrize("dt", [C128, C64], ids=["c128", "c64"])
def test_compare_a_state_with_itself_is_exact(dt):
    n = 18
    psi = rounded(qc.random_state(n, 7), dt)
    h = state_from_host(n, dt, psi)
    try:
        got = sv.sv_compare(h, h)
    finally:
        sv.sv_destroy(h)
    assert got["max_abs"] == 0.0 and got["sq_err"] == 0.0
    assert got["norm_a"] == got["norm_b"]
    assert abs(got["norm_a"] - 1.0) < 1e-6


def test_compare_single_precision_against_double_of_one_circuit():
    """The use it exists for: a complex64 run against the complex128 run of
    the same circuit, within the stated complex64 bound."""
    from tests.gpu_helpers import c64_rel_tol
    n = 20
    g = qc.layer_circuit(n, 10, 4)
    a = sv.sv_create(n, C64)
    b = sv.sv_create(n, C128)
    try:
        sv.sv_run_circuit(a, g, sv.SV_FUSE)
        sv.sv_run_circuit(b, g, sv.SV_FUSE)
        got = sv.sv_compare(a, b)
        host = _numpy_figures(sv.sv_copy_out(a), sv.sv_copy_out(b))
    finally:
        sv.sv_destroy(a)
        sv.sv_destroy(b)
    assert 0 < got["rel_l2"] <= c64_rel_tol(len(g))
    assert got["norm_drift"] <= 1e-5
    assert got["max_abs"] == pytest.approx(host["max_abs"], rel=1e-14)


def test_compare_rejects_mismatched_sizes():
    a = sv.sv_create(5, C128)
    b = sv.sv_create(6, C128)
    try:
        with pytest.raises(sv.SVError) as e:
            sv.sv_compare(a, b)
        assert e.value.status == sv.SV_EINVAL
    finally:
        sv.sv_destroy(a)
        sv.sv_destroy(b)
