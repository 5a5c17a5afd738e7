"""GPU: the uniform initial state and measurement sampling, through the C ABI,
against the oracle and closed forms.

Sampling inverts the CDF of |alpha|^2. The GPU sums in blocks of 4096
amplitudes and the oracle in index order, so the two CDFs differ by rounding:
an index may differ only where the draw u * norm lies within that rounding of
a CDF value between the two indices; everything else must match exactly, and
where probabilities are exact dyadic numbers (the uniform state, even n) every
index must match.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import DTYPE_IDS, DTYPES, assert_close, rounded, state_from_host

pytestmark = pytest.mark.gpu


def _sample(h, u):
    import torch
    ud = torch.as_tensor(np.ascontiguousarray(u, dtype=np.float64)).cuda()
    out = torch.zeros(len(u), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    sv.sv_sample_device(h, ud.data_ptr(), len(u), out.data_ptr())
    sv.sv_synchronize(h)
    return out.cpu().numpy().view(np.uint64)


def _check_against_oracle(psi, u, got, what):
    want = oracle.sample_indices(psi, u)
    p = np.abs(psi) ** 2
    assert (p[got.astype(np.int64)] > 0).all(), f"{what}: drew a zero-probability index"
    bad = np.flatnonzero(got != want)
    cdf = np.cumsum(p)
    norm = cdf[-1]
    for j in bad:
        a, b = sorted((int(got[j]), int(want[j])))
        x = u[j] * norm
        # every CDF value between the two indices is within rounding of the draw
        gap = np.max(np.abs(cdf[a:b] - x))
        assert gap <= 1e-12 * norm, f"{what}: draw {j} gave {got[j]}, oracle {want[j]}"
    assert len(bad) <= max(2, len(u) // 1000), f"{what}: {len(bad)} ambiguous draws"


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [1, 5, 12, 13, 20])
def test_uniform_reset(dtype, n):
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_reset_uniform(h)
        got = sv.sv_copy_out(h)
        ref = np.full(1 << n, oracle.uniform_amplitude(n), dtype=np.complex128)
        assert_close(got, rounded(ref, dtype), dtype, 1, f"uniform n={n}")
        if n % 2 == 0 or dtype == sv.SV_C64:
            assert np.array_equal(got, rounded(ref, dtype))
        # the same state as H on every qubit of |0...0>
        sv.sv_reset(h, 0)
        for q in range(n):
            sv.sv_apply_1q(h, q, qc.H_MATRIX)
        assert_close(sv.sv_copy_out(h), ref, dtype, n, f"H on every qubit n={n}")
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
def test_sampling_a_basis_state(dtype):
    u = qc.sorted_uniforms(11, 5000)
    for n, x in ((3, 5), (12, 4095), (14, 9000), (20, 777777)):
        h = sv.sv_create(n, dtype)
        try:
            sv.sv_reset(h, x)
            assert (_sample(h, u) == x).all(), (n, x)
        finally:
            sv.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [2, 10, 12, 16, 20])
def test_sampling_the_uniform_state_is_exact(dtype, n):
    """Probabilities 2^-n (even n) make every CDF value exact in any order:
    the draw u must give floor(u 2^n)."""
    u = qc.sorted_uniforms(100 + n, 20000)
    h = sv.sv_create(n, dtype)
    try:
        sv.sv_reset_uniform(h)
        got = _sample(h, u)
    finally:
        sv.sv_destroy(h)
    assert np.array_equal(got, np.floor(u * 2.0 ** n).astype(np.uint64))


@pytest.mark.parametrize("dtype", DTYPES, ids=DTYPE_IDS)
@pytest.mark.parametrize("n", [5, 11, 12, 13, 16])
def test_sampling_matches_oracle(dtype, n):
    psi = rounded(qc.random_state(n, 500 + n), dtype)
    u = qc.sorted_uniforms(600 + n, 30000)
    h = state_from_host(n, dtype, psi)
    try:
        got = _sample(h, u)
    finally:
        sv.sv_destroy(h)
    _check_against_oracle(psi, u, got, f"n={n}")


def test_sampling_skips_zero_blocks_and_takes_the_tail():
    """Non-zero amplitudes only in the first of two blocks: draws at the very
    top go to the last non-zero index, not into the empty last block."""
    n = 13
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[[5, 100, 3000]] = [0.6, 0.0, 0.8]
    u = np.array([0.0, 0.2, 0.35, 0.37, 0.5, 0.999999, np.nextafter(1.0, 0.0)])
    h = state_from_host(n, sv.SV_C128, psi)
    try:
        got = _sample(h, u)
    finally:
        sv.sv_destroy(h)
    assert list(got) == list(oracle.sample_indices(psi, u)) == [5, 5, 5, 3000, 3000, 3000, 3000]


def test_sampling_at_24_qubits():
    n = 24
    psi = qc.random_state(n, 2424)
    u = qc.sorted_uniforms(2424, 200000)
    h = state_from_host(n, sv.SV_C128, psi)
    try:
        got = _sample(h, u)
    finally:
        sv.sv_destroy(h)
    _check_against_oracle(psi, u, got, "n=24")
