"""GPU parity at the paper's single-node size (30 qubits) against the CPU
oracle, element by element, through the C ABI.

The fixture `tests/golden/layers30_qft30.npz` was written by
`tests/golden/make_golden_30q.py`, which runs the oracle's stride tier
(Algorithm 1, gate by gate, complex128) on the two 30-qubit circuits the
benchmark times: 20 Haar-SU(2)/CNOT layers from |0...0> (890 gates) and the
QFT of a seeded basis state (465 gates). It holds the amplitudes at 69,000+
seeded indices (random ones, the first 4,096 and a few special ones), the
probabilities of the first 2^16 indices and the norm. Every execution path of
the library runs the same circuits here: gate by gate, fused tile passes with
and without relabelled storage (and with each pass compiled for its own
program, the benchmark's path), and dense 5-qubit blocks; both precisions.

Bounds: complex128 max-abs <= 1e-12 per amplitude; complex64 relative 2-norm
error over the sampled amplitudes <= 8 sqrt(G) 2^-24, G the gates applied.
"""
import os

import numpy as np
import pytest

import paper_1801_01037_amd as sv
from tests.conftest import GOLDEN
from tests.gpu_helpers import C128_MAX_ABS, c64_rel_tol

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(GOLDEN, "layers30_qft30.npz")
MODES = [0, sv.SV_FUSE, sv.SV_FUSE | sv.SV_JIT, sv.SV_FUSE | sv.SV_NO_RELABEL, sv.SV_FUSE_DENSE]
MODE_IDS = ["per-gate", "fused", "fused-compiled", "fused-standard-order", "dense"]


@pytest.fixture(scope="module")
def gold():
    with np.load(FIXTURE) as z:   # plain arrays only (no pickles)
        return {k: z[k] for k in z.files}


def _circuit(which, gold):
    import qcircuits as qc
    n = int(gold["n"])
    if which == "layers":
        g, x = qc.layer_circuit(n, 20, 1), 0
    else:
        g, x = qc.qft_circuit(n), int(gold["qft_x"])
    assert len(g) == int(gold[f"{which}_gates"])
    return n, g, x


def _gather(st, idx):
    import torch
    t = torch.from_numpy(idx).to(st.tensor.device)
    return st.tensor[t].cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("flags", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dtype", [sv.SV_C128, sv.SV_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("which", ["layers", "qft"])
def test_30_qubits_against_oracle(gold, which, dtype, flags):
    n, g, x = _circuit(which, gold)
    idx = gold["indices"]
    ref = gold[f"{which}_amp"]
    pref = gold[f"{which}_probs"]
    print(f"{which} n={n} dtype={dtype} flags={flags} gates={len(g)}", flush=True)
    with sv.StateVector(n, dtype, basis_index=x) as st:
        st.run(g, flags)
        got = _gather(st, idx)
        probs = sv.sv_probs(st.handle, 0, len(pref))
        nrm = st.norm()
    if dtype == sv.SV_C128:
        err = float(np.max(np.abs(got - ref)))
        print(f"  max-abs {err:.3e}", flush=True)
        assert err <= C128_MAX_ABS
        # |p - p_ref| <= 2 |alpha| d + d^2 for an amplitude error d <= 1e-12
        amp = np.sqrt(pref)
        assert np.all(np.abs(probs - pref) <= 2 * amp * C128_MAX_ABS + C128_MAX_ABS ** 2)
        assert abs(nrm - float(gold[f"{which}_norm"])) <= 1e-12
    else:
        rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        tol = c64_rel_tol(len(g))
        print(f"  rel 2-norm {rel:.3e} (bound {tol:.3e}), max-abs "
              f"{float(np.max(np.abs(got - ref))):.3e}", flush=True)
        assert rel <= tol
        prel = float(np.linalg.norm(probs - pref) / np.linalg.norm(pref))
        assert prel <= 2 * tol
        assert abs(nrm - 1.0) <= 1e-5
