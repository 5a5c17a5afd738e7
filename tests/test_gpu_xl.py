"""The 33-qubit complex128 and 34-qubit complex64 registers (128 GiB each): the
paper's largest run (33 qubits over 64 nodes) on one GPU.

No host oracle can step these states inside a test, so the checks are the
ones that hold at any size, with sampled amplitudes where a closed form
exists: the QFT of a basis state against its closed form, and the depth-10
random circuit followed by its adjoint returning to the start state, for the
dense-block, tile and per-gate paths (per-gate only in complex64, to bound
the test time).
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
