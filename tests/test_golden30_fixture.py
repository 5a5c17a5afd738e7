"""The 30-qubit oracle fixture (tests/golden/layers30_qft30.npz) on the CPU:
its indices are the generator's, its QFT amplitudes are the closed form for
the QFT of a basis state, and both stored states have norm one. The fixture is
written only by tests/golden/make_golden_30q.py, which calls the oracle."""
import os

import numpy as np

import oracle
from tests.conftest import GOLDEN
from tests.golden.make_golden_30q import N, N_PROBS, sample_indices

FIXTURE = os.path.join(GOLDEN, "layers30_qft30.npz")


def _load():
    with np.load(FIXTURE) as z:   # plain arrays only (no pickles)
        return {k: z[k] for k in z.files}


def test_fixture_indices_and_shapes():
    g = _load()
    assert int(g["n"]) == N
    assert np.array_equal(g["indices"], sample_indices())
    for w in ("layers", "qft"):
        assert g[f"{w}_amp"].shape == g["indices"].shape
        assert g[f"{w}_amp"].dtype == np.complex128
        assert g[f"{w}_probs"].shape == (N_PROBS,)
        assert abs(float(g[f"{w}_norm"]) - 1.0) <= 1e-12


def test_fixture_qft_is_the_closed_form():
    g = _load()
    some = g["indices"][::97]
    closed = oracle.qft_basis_amplitudes(N, int(g["qft_x"]), some)
    assert np.max(np.abs(g["qft_amp"][::97] - closed)) <= 1e-12
    # |alpha|^2 = 2^-30 everywhere for the QFT of a basis state
    assert np.max(np.abs(g["qft_probs"] - 2.0 ** -N)) <= 1e-12 * 2.0 ** -N


def test_fixture_probs_agree_with_stored_amplitudes():
    g = _load()
    idx = g["indices"]
    lead = idx < N_PROBS
    amp = g["layers_amp"][lead]
    p = g["layers_probs"][idx[lead]]
    assert np.array_equal(p, amp.real * amp.real + amp.imag * amp.imag)
