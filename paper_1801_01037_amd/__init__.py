"""MI355X state-vector simulator: a thin ctypes binding of libsv.so.

Every function here has the name and meaning of the C entry point declared in
include/sv.h and only marshals arguments; all state work runs in the HIP
kernels of libsv.so. There is no CPU fallback: if the library is missing the
import of any entry point raises.

`StateVector` is a convenience wrapper that takes its device memory and stream
from PyTorch (torch.complex64 / torch.complex128 tensors on the GPU) and
passes them to sv_wrap.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "SV_C64", "SV_C128", "SV_FUSE", "SV_FUSE_DENSE", "SV_GRAPH", "SV_NO_RELABEL", "SV_JIT", "SVError", "lib",
    "sv_version", "sv_last_error", "sv_create", "sv_wrap", "sv_destroy", "sv_set_stream",
    "sv_set_tile_geometry",
    "sv_info", "sv_reset", "sv_reset_uniform", "sv_sample_device", "sv_sample_device_noalloc", "sv_apply_1q", "sv_apply_ctrl", "sv_apply_mcu", "sv_apply_unitary", "sv_apply_cphase",
    "sv_run_circuit", "sv_run_circuit_ex", "sv_run_batch", "sv_probs", "sv_probs_device", "sv_norm", "sv_norm_device", "sv_compare",
    "sv_copy_out", "sv_copy_in", "sv_synchronize", "sv_profile", "sv_profile_read",
    "sv_plan_inspect", "sv_plan_dense_inspect", "sv_plan_jit_check", "sv_plan_create", "sv_plan_destroy",
    "sv_plan_passes", "sv_run_plan", "sv_batch_create", "sv_batch_destroy", "sv_batch_config",
    "sv_batch_persist", "sv_batch_solo", "sv_batch_run", "sv_batch_times", "StateVector", "LIB_PATH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsv.so")

SV_C64 = 1
SV_C128 = 2
SV_FUSE = 1
SV_FUSE_DENSE = 2
SV_GRAPH = 4
SV_NO_RELABEL = 8
SV_JIT = 16

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, -1, -2, -3, -4
_STATUS_NAMES = {SV_EINVAL: "SV_EINVAL", SV_ENOMEM: "SV_ENOMEM",
                 SV_EDEVICE: "SV_EDEVICE", SV_EUNSUPPORTED: "SV_EUNSUPPORTED"}

GATE_DTYPE = np.dtype([
    ("kind", "<i4"), ("control", "<i4"), ("target", "<i4"), ("flags", "<i4"),
    ("m", "<f8", (8,)),
])


class SVError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


_lib = None
_vp, _u64, _int, _u32, _sz = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                              ctypes.c_uint32, ctypes.c_size_t)
_dp = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "sv_version": ([], ctypes.c_int),
    "sv_last_error": ([], ctypes.c_char_p),
    "sv_create": ([_int, _int, _vp, ctypes.POINTER(_vp)], _int),
    "sv_wrap": ([_vp, _int, _int, _vp, ctypes.POINTER(_vp)], _int),
    "sv_destroy": ([_vp], _int),
    "sv_set_stream": ([_vp, _vp], _int),
    "sv_set_tile_geometry": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], _int),
    "sv_info": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_int), ctypes.POINTER(_int)], _int),
    "sv_reset": ([_vp, _u64], _int),
    "sv_apply_1q": ([_vp, _int, _dp], _int),
    "sv_apply_ctrl": ([_vp, _int, _int, _dp], _int),
    "sv_apply_mcu": ([_vp, ctypes.c_uint64, _int, _dp], _int),
    "sv_apply_unitary": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _dp], _int),
    "sv_reset_uniform": ([_vp], _int),
    "sv_sample_device": ([_vp, _vp, ctypes.c_uint64, _vp], _int),
    "sv_sample_device_noalloc": ([_vp, _vp, ctypes.c_uint64, _vp], _int),
    "sv_apply_cphase": ([_vp, _int, _int, ctypes.c_double], _int),
    "sv_run_circuit": ([_vp, _vp, _sz, _u32], _int),
    "sv_run_circuit_ex": ([_vp, _vp, _sz, _vp, _sz, _u32], _int),
    "sv_run_batch": ([_vp, _vp, _vp, _sz, _u32], _int),
    "sv_probs": ([_vp, _u64, _u64, _dp], _int),
    "sv_probs_device": ([_vp, _u64, _u64, _vp], _int),
    "sv_norm": ([_vp, _dp], _int),
    "sv_norm_device": ([_vp, _vp], _int),
    "sv_compare": ([_vp, _vp, _dp], _int),
    "sv_copy_out": ([_vp, _vp], _int),
    "sv_copy_in": ([_vp, _vp], _int),
    "sv_synchronize": ([_vp], _int),
    "sv_profile": ([_vp, _int], _int),
    "sv_plan_inspect": ([_int, _int, _vp, _sz, _u32, _vp, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], _int),
    "sv_plan_dense_inspect": ([_int, _vp, _sz, _vp, _vp, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32)], _int),
    "sv_plan_jit_check": ([_int, _int, _vp, _sz, _u32, ctypes.POINTER(ctypes.c_int32)], _int),
    "sv_plan_create": ([_vp, _vp, _sz, ctypes.POINTER(_vp)], _int),
    "sv_plan_destroy": ([_vp], _int),
    "sv_plan_passes": ([_vp, ctypes.POINTER(ctypes.c_int32)], _int),
    "sv_run_plan": ([_vp, ctypes.c_int32, ctypes.c_int32], _int),
    "sv_batch_create": ([_int, _vp, ctypes.POINTER(_vp)], _int),
    "sv_batch_destroy": ([_vp], _int),
    "sv_batch_config": ([_vp, ctypes.c_int32, ctypes.c_int32], _int),
    "sv_batch_persist": ([_vp, ctypes.c_int32], _int),
    "sv_batch_solo": ([_vp, ctypes.c_int32], _int),
    "sv_batch_run": ([_vp, _vp, _vp, _vp, _sz, _u32], _int),
    "sv_batch_times": ([_vp, _dp, _dp, _sz], _int),
    "sv_profile_read": ([_vp, ctypes.POINTER(_ProfEntry), _int, ctypes.POINTER(_int)], _int),
}


def lib():
    """The loaded libsv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_1801_01037_amd/build.py` (there is no fallback)")
        # PyTorch ships its own HIP runtime under a file name the system one
        # does not satisfy. Loading torch first makes libsv's libamdhip64.so.7
        # resolve to that already-loaded runtime, so the process holds one HIP
        # runtime whichever of the two is used first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != SV_OK:
        raise SVError(status, sv_last_error())


def _mat(m) -> ctypes.Array:
    a = np.ascontiguousarray(m, dtype=np.float64)
    if a.shape != (8,):
        raise ValueError("a gate matrix is 8 doubles: q11, q12, q21, q22 as (re, im)")
    return (ctypes.c_double * 8)(*a.tolist())


def sv_version() -> int:
    return lib().sv_version()


def sv_last_error() -> str:
    return lib().sv_last_error().decode()


def sv_create(n_qubits: int, dtype: int, stream: int | None = None) -> int:
    h = _vp()
    _check(lib().sv_create(n_qubits, dtype, stream, ctypes.byref(h)))
    return h.value


def sv_wrap(dev_ptr: int, n_qubits: int, dtype: int, stream: int | None = None) -> int:
    h = _vp()
    _check(lib().sv_wrap(dev_ptr, n_qubits, dtype, stream, ctypes.byref(h)))
    return h.value


def sv_destroy(h: int) -> None:
    _check(lib().sv_destroy(h))


def sv_set_stream(h: int, stream: int | None) -> None:
    _check(lib().sv_set_stream(h, stream))


def sv_set_tile_geometry(h: int, tile_qubits: int = 0, register_qubits: int = 0,
                         low_qubits: int = -1) -> None:
    """Tile geometry of the handle's SV_FUSE runs and plans (0 / 0 / -1:
    defaults; see include/sv.h)."""
    _check(lib().sv_set_tile_geometry(h, tile_qubits, register_qubits, low_qubits))


def sv_info(h: int):
    p, n, dt = _vp(), _int(), _int()
    _check(lib().sv_info(h, ctypes.byref(p), ctypes.byref(n), ctypes.byref(dt)))
    return p.value, n.value, dt.value


def sv_reset(h: int, basis_index: int = 0) -> None:
    _check(lib().sv_reset(h, basis_index))


def sv_reset_uniform(h: int) -> None:
    _check(lib().sv_reset_uniform(h))


def sv_sample_device(h: int, u_dev: int, count: int, out_dev: int) -> None:
    """Device pointers: `count` ascending doubles in [0, 1) in, `count` uint64
    indices out (see include/sv.h)."""
    _check(lib().sv_sample_device(h, u_dev, count, out_dev))


def sv_sample_device_noalloc(h: int, u_dev: int, count: int, out_dev: int) -> None:
    """As sv_sample_device, with the library's static scratch (n <= 30; no
    allocation of any kind)."""
    _check(lib().sv_sample_device_noalloc(h, u_dev, count, out_dev))


def sv_apply_1q(h: int, target: int, m) -> None:
    _check(lib().sv_apply_1q(h, target, _mat(m)))


def sv_apply_ctrl(h: int, control: int, target: int, m) -> None:
    _check(lib().sv_apply_ctrl(h, control, target, _mat(m)))


def sv_apply_mcu(h: int, controls, target: int, m) -> None:
    """2x2 gate on `target` where every qubit of `controls` is 1 (Toffoli:
    two controls, m = X)."""
    mask = 0
    for c in controls:
        mask |= 1 << int(c)
    _check(lib().sv_apply_mcu(h, mask, target, _mat(m)))


def sv_apply_unitary(h: int, qubits, u) -> None:
    """General gate: the 2^k x 2^k complex matrix u on `qubits` (k <= 5),
    qubits[0] the least significant bit of the local index."""
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(u, dtype=np.complex128)
    if m.shape != (1 << len(q), 1 << len(q)):
        raise ValueError("u must be 2^k x 2^k for k qubits")
    _check(lib().sv_apply_unitary(h, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(q),
                                  m.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def sv_apply_cphase(h: int, control: int, target: int, theta: float) -> None:
    _check(lib().sv_apply_cphase(h, control, target, float(theta)))


def sv_run_circuit(h: int, gates: np.ndarray, flags: int = 0, mats=None) -> None:
    """Runs a gate list; `mats` (qcircuits.unitary_table) is the matrix table of
    its SV_G_UNITARY records, if any (sv_run_circuit_ex)."""
    g = _gates(gates)
    ptr = g.ctypes.data if len(g) else None
    if mats is None:
        _check(lib().sv_run_circuit(h, ptr, len(g), flags))
        return
    t = np.ascontiguousarray(mats, dtype=np.float64)
    if t.ndim != 2 or t.shape[1] != 2048:
        raise ValueError("mats: one row of 2048 doubles per matrix")
    _check(lib().sv_run_circuit_ex(h, ptr, len(g), t.ctypes.data if len(t) else None, len(t), flags))


def sv_run_batch(handles, circuits, flags: int = 0) -> None:
    """Runs circuits[c] on handles[c] for every c as one batch (synchronous)."""
    if len(handles) != len(circuits):
        raise ValueError("one circuit per state")
    arrs = []
    for gates in circuits:
        g = np.ascontiguousarray(gates)
        arrs.append(g if g.dtype == GATE_DTYPE else g.astype(GATE_DTYPE))
    k = len(arrs)
    hs = (ctypes.c_void_p * max(k, 1))(*handles)
    ps = (ctypes.c_void_p * max(k, 1))(*[g.ctypes.data if len(g) else None for g in arrs])
    ls = (ctypes.c_size_t * max(k, 1))(*[len(g) for g in arrs])
    _check(lib().sv_run_batch(hs, ps, ls, k, flags))


def sv_probs(h: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _check(lib().sv_probs(h, first, count, out.ctypes.data_as(_dp)))
    return out


def sv_probs_device(h: int, first: int, count: int, out_dev: int) -> None:
    _check(lib().sv_probs_device(h, first, count, out_dev))


def sv_norm(h: int) -> float:
    v = ctypes.c_double()
    _check(lib().sv_norm(h, ctypes.byref(v)))
    return v.value


def sv_norm_device(h: int, out_dev: int) -> None:
    _check(lib().sv_norm_device(h, out_dev))


def sv_compare(a: int, b: int) -> dict:
    """State a against state b in FP64 on the GPU: max-abs amplitude error,
    sum |a - b|^2, both norms, and the derived relative 2-norm error and a's
    norm drift (see include/sv.h)."""
    out = np.zeros(4, dtype=np.float64)
    _check(lib().sv_compare(a, b, out.ctypes.data_as(_dp)))
    mx, d2, na, nb = (float(v) for v in out)
    return {"max_abs": mx, "sq_err": d2, "norm_a": na, "norm_b": nb,
            "rel_l2": (d2 / nb) ** 0.5 if nb > 0 else float("nan"),
            "norm_drift": abs(na - 1.0)}


def sv_copy_out(h: int) -> np.ndarray:
    _, n, dt = sv_info(h)
    out = np.empty(1 << n, dtype=np.complex64 if dt == SV_C64 else np.complex128)
    _check(lib().sv_copy_out(h, out.ctypes.data))
    return out


def sv_copy_in(h: int, host: np.ndarray) -> None:
    _, n, dt = sv_info(h)
    want = np.complex64 if dt == SV_C64 else np.complex128
    a = np.ascontiguousarray(host, dtype=want)
    if a.size != 1 << n:
        raise ValueError(f"expected {1 << n} amplitudes, got {a.size}")
    _check(lib().sv_copy_in(h, a.ctypes.data))


def sv_synchronize(h: int) -> None:
    _check(lib().sv_synchronize(h))


def sv_profile(h: int, enable: bool) -> None:
    _check(lib().sv_profile(h, 1 if enable else 0))


def sv_profile_read(h: int) -> dict:
    """{kernel class: {launches, total_ms, bytes, flops}} of the timed launches."""
    buf = (_ProfEntry * 16)()
    cnt = _int()
    _check(lib().sv_profile_read(h, buf, 16, ctypes.byref(cnt)))
    return {e.name.decode(): {"launches": int(e.launches), "total_ms": e.total_ms,
                              "bytes": e.bytes, "flops": e.flops}
            for e in buf[:min(cnt.value, 16)]}


def sv_plan_inspect(n_qubits: int, dtype: int, gates: np.ndarray, flags: int = SV_FUSE):
    """Host-only plan of a gate list: (gate_op array, n_passes, n_groups, n_ops)."""
    g = np.ascontiguousarray(gates)
    if g.dtype != GATE_DTYPE:
        g = g.astype(GATE_DTYPE)
    gate_op = np.empty(len(g), dtype=np.int32)
    p, gr, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sv_plan_inspect(n_qubits, dtype, g.ctypes.data if len(g) else None, len(g),
                                 flags, gate_op.ctypes.data, ctypes.byref(p), ctypes.byref(gr),
                                 ctypes.byref(o)))
    return gate_op, p.value, gr.value, o.value


def sv_plan_dense_inspect(n_qubits: int, gates: np.ndarray, cap: int | None = None):
    """Host-only dense-block plan: (block masks, complex (nb, 32, 32) matrices)."""
    g = np.ascontiguousarray(gates)
    if g.dtype != GATE_DTYPE:
        g = g.astype(GATE_DTYPE)
    nb = ctypes.c_int32()
    ptr = g.ctypes.data if len(g) else None
    _check(lib().sv_plan_dense_inspect(n_qubits, ptr, len(g), None, None, 0, ctypes.byref(nb)))
    cap = nb.value if cap is None else min(cap, nb.value)
    masks = np.zeros(cap, dtype=np.uint64)
    mats = np.zeros((cap, 32, 32), dtype=np.complex128)
    _check(lib().sv_plan_dense_inspect(n_qubits, ptr, len(g), masks.ctypes.data, mats.ctypes.data,
                                       cap, ctypes.byref(nb)))
    return masks, mats


def sv_plan_jit_check(n_qubits: int, dtype: int, gates: np.ndarray,
                      flags: int = SV_FUSE | SV_JIT) -> int:
    """Host only: compiles the pass programs SV_FUSE | SV_JIT would run for
    this gate list; returns their number (see include/sv.h)."""
    g = _gates(gates)
    nprog = ctypes.c_int32()
    _check(lib().sv_plan_jit_check(n_qubits, dtype, g.ctypes.data if len(g) else None, len(g),
                                   flags, ctypes.byref(nprog)))
    return nprog.value


def _gates(gates):
    g = np.ascontiguousarray(gates)
    if g.dtype != GATE_DTYPE:
        g = g.astype(GATE_DTYPE)
    return g


def sv_plan_create(h: int, gates: np.ndarray) -> int:
    g = _gates(gates)
    p = _vp()
    _check(lib().sv_plan_create(h, g.ctypes.data if len(g) else None, len(g), ctypes.byref(p)))
    return p.value


def sv_plan_destroy(p: int) -> None:
    _check(lib().sv_plan_destroy(p))


def sv_plan_passes(p: int) -> int:
    v = ctypes.c_int32()
    _check(lib().sv_plan_passes(p, ctypes.byref(v)))
    return v.value


def sv_run_plan(p: int, first_pass: int, count: int) -> None:
    _check(lib().sv_run_plan(p, first_pass, count))


def sv_batch_create(dtype: int, stream: int | None = None) -> int:
    b = _vp()
    _check(lib().sv_batch_create(dtype, stream, ctypes.byref(b)))
    return b.value


def sv_batch_destroy(b: int) -> None:
    _check(lib().sv_batch_destroy(b))


def sv_batch_persist(b: int, max_tiles: int) -> None:
    """Circuits of at most max_tiles tiles per pass run whole in one persistent
    launch (0: off)."""
    _check(lib().sv_batch_persist(b, int(max_tiles)))


def sv_batch_solo(b: int, min_tiles: int) -> None:
    """Circuits of at least min_tiles tiles per pass run pass by pass on a
    third stream, beside the levels (0: off)."""
    _check(lib().sv_batch_solo(b, int(min_tiles)))


def sv_batch_config(b: int, blocks_per_cu: int, tiles_per_task: int) -> None:
    _check(lib().sv_batch_config(b, blocks_per_cu, tiles_per_task))


def sv_batch_run(b: int, plans, first_pass=None, pass_count=None, flags: int = 0) -> None:
    n = len(plans)
    arr = (_vp * max(n, 1))(*plans)
    fp = None if first_pass is None else np.ascontiguousarray(first_pass, dtype=np.int32)
    pc = None if pass_count is None else np.ascontiguousarray(pass_count, dtype=np.int32)
    _check(lib().sv_batch_run(b, arr, None if fp is None else fp.ctypes.data,
                              None if pc is None else pc.ctypes.data, n, flags))


def sv_batch_times(b: int, count: int):
    """(start_ms, end_ms) per circuit of the last run (device clock, waits)."""
    st = np.zeros(count)
    en = np.zeros(count)
    _check(lib().sv_batch_times(b, st.ctypes.data_as(_dp), en.ctypes.data_as(_dp), count))
    return st, en


class StateVector:
    """A state whose device memory is a torch tensor, driven through libsv."""

    def __init__(self, n_qubits: int, dtype: int = SV_C128, device: int = 0,
                 stream=None, basis_index: int = 0):
        import torch
        tdt = torch.complex64 if dtype == SV_C64 else torch.complex128
        self.n, self.dtype = n_qubits, dtype
        self.tensor = torch.empty(1 << n_qubits, dtype=tdt, device=f"cuda:{device}")
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        self.handle = sv_wrap(self.tensor.data_ptr(), n_qubits, dtype, s.cuda_stream)
        sv_reset(self.handle, basis_index)

    def reset(self, basis_index: int = 0):
        sv_reset(self.handle, basis_index)

    def apply_1q(self, target, m):
        sv_apply_1q(self.handle, target, m)

    def apply_ctrl(self, control, target, m):
        sv_apply_ctrl(self.handle, control, target, m)

    def apply_mcu(self, controls, target, m):
        sv_apply_mcu(self.handle, controls, target, m)

    def apply_unitary(self, qubits, u):
        sv_apply_unitary(self.handle, qubits, u)

    def apply_cphase(self, control, target, theta):
        sv_apply_cphase(self.handle, control, target, theta)

    def set_tile_geometry(self, tile_qubits: int = 0, register_qubits: int = 0,
                          low_qubits: int = -1):
        sv_set_tile_geometry(self.handle, tile_qubits, register_qubits, low_qubits)

    def run(self, gates, flags: int = 0, mats=None):
        sv_run_circuit(self.handle, gates, flags, mats)

    def probs(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        return sv_probs(self.handle, first, count)

    def reset_uniform(self):
        sv_reset_uniform(self.handle)

    def sample(self, u) -> np.ndarray:
        """Basis indices drawn by the uniforms `u` (ascending, in [0, 1))."""
        import torch
        with torch.cuda.stream(self.stream):   # copies ordered with the handle's work
            ud = torch.as_tensor(np.ascontiguousarray(u, dtype=np.float64)).to(self.tensor.device)
            out = torch.empty(len(ud), dtype=torch.int64, device=self.tensor.device)
            if len(ud):
                sv_sample_device(self.handle, ud.data_ptr(), len(ud), out.data_ptr())
            host = out.cpu()
        self.synchronize()
        return host.numpy().view(np.uint64)

    def norm(self) -> float:
        return sv_norm(self.handle)

    def numpy(self) -> np.ndarray:
        return sv_copy_out(self.handle)

    def synchronize(self):
        sv_synchronize(self.handle)

    def close(self):
        if self.handle:
            sv_destroy(self.handle)
            self.handle = None
            self.tensor = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
