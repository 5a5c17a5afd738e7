"""The C ABI on the CPU: the library loads, exports every declared entry point,
and rejects bad arguments before it touches a device."""
import ctypes
import os
import re

import pytest

import paper_1801_01037_amd as sv

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "sv.h")


def _declared():
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sv.LIB_PATH):
        import paper_1801_01037_amd.build as b
        b.build()
    return sv.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "sv_create" in names and "sv_run_circuit" in names and "sv_probs" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(sv.__all__), set(names) - set(sv.__all__)


def test_version(lib):
    assert sv.sv_version() == 3


def test_rejects_bad_arguments_without_a_device(lib):
    h = ctypes.c_void_p()
    assert lib.sv_create(0, sv.SV_C128, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert "n_qubits" in sv.sv_last_error()
    assert lib.sv_create(35, sv.SV_C64, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert lib.sv_create(10, 7, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert lib.sv_create(10, sv.SV_C64, None, None) == sv.SV_EINVAL
    assert lib.sv_wrap(None, 10, sv.SV_C64, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert lib.sv_wrap(8, 10, sv.SV_C64, None, ctypes.byref(h)) == sv.SV_EINVAL  # misaligned
    assert lib.sv_destroy(None) == sv.SV_OK
    assert lib.sv_set_tile_geometry(None, 0, 0, -1) == sv.SV_EINVAL
    assert lib.sv_reset(None, 0) == sv.SV_EINVAL
    assert lib.sv_run_circuit(None, None, 1, 0) == sv.SV_EINVAL
    assert lib.sv_run_batch(None, None, None, 1, 0) == sv.SV_EINVAL
    assert lib.sv_run_batch(None, None, None, 0, 0) == sv.SV_OK
    one = (ctypes.c_void_p * 1)(None)
    lens = (ctypes.c_size_t * 1)(0)
    assert lib.sv_run_batch(one, one, lens, 1, 0x100) == sv.SV_EINVAL
    assert "flags" in sv.sv_last_error()
    assert lib.sv_run_batch(one, one, lens, 1, sv.SV_FUSE) == sv.SV_EINVAL   # null state
    assert lib.sv_batch_solo(None, 4) == sv.SV_EINVAL
    assert lib.sv_norm(None, None) == sv.SV_EINVAL
    assert lib.sv_synchronize(None) == sv.SV_EINVAL
    with pytest.raises(sv.SVError) as ei:
        sv.sv_reset(None, 0)
    assert ei.value.status == sv.SV_EINVAL


def test_gate_record_layout_matches_header():
    import qcircuits as qc
    assert sv.GATE_DTYPE == qc.GATE_DTYPE
    assert sv.GATE_DTYPE.itemsize == 80
    assert [sv.GATE_DTYPE.fields[k][1] for k in ("kind", "control", "target", "flags", "m")] \
        == [0, 4, 8, 12, 16]
