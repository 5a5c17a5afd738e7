"""The 33-qubit complex128 and 34-qubit complex64 registers (128 GiB each): the
paper's largest run (33 qubits over 64 nodes) on one GPU.

No host oracle can step these states inside a test, so the checks are the
ones that hold at any size, with sampled amplitudes where a closed form
exists: the QFT of a basis state against its closed form, the depth-10
random circuit followed by its adjoint returning to the start state (dense-block
and tile paths), and gate by gate a Hadamard on every qubit, controlled phases
and a controlled sequence with its adjoint, each against the closed form.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import C128_MAX_ABS, c64_rel_tol

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28


def _max_abs_except(t, x):
    """max |t[i]| over i != x, in chunks (no state-sized temporaries)."""
    import torch
    saved = t[x].clone()
    t[x] = 0
    m = 0.0
    for lo in range(0, t.numel(), CHUNK):
        m = max(m, t[lo:lo + CHUNK].abs().max().item())
    t[x] = saved
    torch.cuda.synchronize()
    return m


def _sample(n, seed, count=2048):
    r = qc.splitmix64(seed, count) >> np.uint64(64 - n)
    return np.unique(np.concatenate([r, np.array([0, (1 << n) - 1], dtype=np.uint64)])).astype(np.int64)


CASES = [(33, sv.SV_C128), (34, sv.SV_C64)]
IDS = ["33q-c128", "34q-c64"]


@pytest.mark.parametrize("n,dtype", CASES, ids=IDS)
@pytest.mark.parametrize("flags", [sv.SV_FUSE, sv.SV_FUSE_DENSE], ids=["tile", "dense"])
def test_mirror_largest_register(n, dtype, flags):
    g = qc.layer_circuit(n, 10, 5)
    x = qc.random_basis_index(n, 6)
    with sv.StateVector(n, dtype, basis_index=x) as st:
        st.run(g, flags)
        mid = st.norm()
        st.run(qc.inverse_circuit(g), flags)
        at_x = complex(st.tensor[x].item())
        rest = _max_abs_except(st.tensor, x)
    if dtype == sv.SV_C128:
        assert abs(at_x - 1) <= C128_MAX_ABS and rest <= C128_MAX_ABS
        assert abs(mid - 1) <= 1e-12
    else:
        tol = c64_rel_tol(2 * len(g))
        assert abs(at_x - 1) <= tol and rest <= tol
        assert abs(mid - 1) <= 1e-5


@pytest.mark.parametrize("n,dtype", CASES, ids=IDS)
def test_qft_largest_register(n, dtype):
    import torch
    x = qc.random_basis_index(n, 8)
    idx = _sample(n, 9)
    ref = oracle.qft_basis_amplitudes(n, x, idx)
    with sv.StateVector(n, dtype, basis_index=x) as st:
        st.run(qc.qft_circuit(n), sv.SV_FUSE)
        got = st.tensor[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
        nrm = st.norm()
    if dtype == sv.SV_C128:
        assert np.max(np.abs(got - ref)) <= C128_MAX_ABS
        assert abs(nrm - 1) <= 1e-12
    else:
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= c64_rel_tol(n * (n + 1) // 2)
        assert abs(nrm - 1) <= 1e-5


@pytest.mark.parametrize("n,dtype", CASES, ids=IDS)
def test_per_gate_layouts_largest_register(n, dtype):
    """Gate by gate at 2^33 / 2^34 amplitudes (more work-items than one launch
    holds at one per thread): H on every qubit gives the uniform state; phases
    on (0, 1), (0, n-1), (2, 5), (14, 15) give e^{i sum theta} on the indices
    with both bits set; controlled gates with controls inside and above the
    128-byte line, followed by their adjoint, give that state back."""
    import math
    import torch
    idx = _sample(n, 31)
    tidx = torch.from_numpy(idx).cuda()
    h = qc.H_MATRIX
    cps = [(0, 1, 0.3), (0, n - 1, 0.7), (2, 5, 1.1), (14, 15, 1.9)]
    u = qc.haar_su2(3300 + n, 4)
    ctl = np.concatenate([qc.gate_cu(0, n - 1, u[0]), qc.gate_cu(n - 1, 1, u[1]),
                          qc.gate_cnot(2, 20), qc.gate_mcu((0, 1, 2), n - 1, qc.X_MATRIX),
                          qc.gate_mcu((1, n - 2), 3, u[2]), qc.gate_cu(5, 0, u[3])])
    amp = 2.0 ** (-n / 2)
    ph = np.zeros(len(idx))
    for c, t, th in cps:
        ph += np.where(((idx >> c) & 1) & ((idx >> t) & 1) == 1, th, 0.0)
    want = amp * np.exp(1j * ph)
    with sv.StateVector(n, dtype) as st:
        for q in range(n):
            st.apply_1q(q, h)
        uni = st.tensor[tidx].cpu().numpy().astype(np.complex128)
        for c, t, th in cps:
            st.apply_cphase(c, t, th)
        mid = st.tensor[tidx].cpu().numpy().astype(np.complex128)
        st.run(ctl, 0)
        moved = st.tensor[tidx].cpu().numpy().astype(np.complex128)
        st.run(qc.inverse_circuit(ctl), 0)
        back = st.tensor[tidx].cpu().numpy().astype(np.complex128)
        nrm = st.norm()
    assert np.max(np.abs(moved - want)) > 1e-3 * amp      # the controlled gates did act
    if dtype == sv.SV_C128:
        assert np.max(np.abs(uni - amp)) <= C128_MAX_ABS * amp
        for got in (mid, back):
            assert np.max(np.abs(got - want)) <= C128_MAX_ABS * amp
        assert abs(nrm - 1) <= 1e-12
    else:
        for got, k in ((uni, n), (mid, n + 4), (back, n + 4 + 2 * len(ctl))):
            ref = want if got is not uni else np.full(len(idx), amp)
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= c64_rel_tol(k)
        assert abs(nrm - 1) <= 1e-5
    assert math.isfinite(nrm)
