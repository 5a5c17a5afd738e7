"""Writes the 30-qubit reference fixture `layers30_qft30.npz` from the CPU oracle.

The fixture holds what the oracle's stride tier (Algorithm 1, gate by gate, in
complex128) gives for the two 30-qubit circuits the benchmark runs:
  * `layer_circuit(30, 20, 1)` from |0...0>: 20 layers of a Haar SU(2) on every
    qubit followed by CNOTs on neighbour pairs (600 + 290 gates);
  * `qft_circuit(30)` from |x>, x = random_basis_index(30, 2024) (465 gates).
Stored for each: the amplitudes at a seeded sample of indices (65,536 drawn
from SplitMix64 plus the first 4,096 indices and a few special ones), the
probabilities |alpha_i|^2 of the first 2^16 indices, and the FP64 norm.

Only `oracle/` and the seeded input generators of `qcircuits/` are called. The
QFT result is also checked here against the oracle's closed form for the QFT
of a basis state at every stored index before anything is written.

Run:  python tests/golden/make_golden_30q.py [threads]
(about 16 GiB of host memory per state; some minutes with 8 threads)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import qcircuits as qc  # noqa: E402

N = 30
DEPTH = 20
LAYER_SEED = 1
QFT_X_SEED = 2024
INDEX_SEED = 0x30D20
N_RANDOM = 1 << 16
N_LEADING = 1 << 12
N_PROBS = 1 << 16
OUT = os.path.join(HERE, "layers30_qft30.npz")


def sample_indices(n: int = N) -> np.ndarray:
    """The stored indices: seeded random ones, the leading block and a few
    special ones, sorted and without repeats."""
    r = (qc.splitmix64(INDEX_SEED, N_RANDOM) >> np.uint64(64 - n)).astype(np.int64)
    lead = np.arange(N_LEADING, dtype=np.int64)
    top = (1 << n) - 1
    special = np.array([top, 1 << (n - 1), top ^ 1, 0x2AAAAAAA & top, 0x15555555 & top],
                       dtype=np.int64)
    return np.unique(np.concatenate([r, lead, special]))


def _run(n, gates, x, threads):
    t = time.time()
    psi = oracle.basis_state(n, x)
    oracle.run_circuit(psi, gates)
    print(f"  {len(gates)} gates in {time.time() - t:.0f} s ({threads} threads)", flush=True)
    return psi


def main(threads: int) -> None:
    used = oracle.set_threads(threads)
    idx = sample_indices()
    out = {"indices": idx, "n": np.int64(N)}

    print("layers: depth 20, seed 1, from |0>", flush=True)
    g = qc.layer_circuit(N, DEPTH, LAYER_SEED)
    psi = _run(N, g, 0, used)
    out["layers_amp"] = psi[idx].copy()
    out["layers_probs"] = oracle.probs(psi, 0, N_PROBS)
    out["layers_norm"] = np.float64(oracle.norm(psi))
    out["layers_gates"] = np.int64(len(g))
    del psi

    x = qc.random_basis_index(N, QFT_X_SEED)
    print(f"qft from |{x}>", flush=True)
    g = qc.qft_circuit(N)
    psi = _run(N, g, x, used)
    amp = psi[idx].copy()
    out["qft_amp"] = amp
    out["qft_probs"] = oracle.probs(psi, 0, N_PROBS)
    out["qft_norm"] = np.float64(oracle.norm(psi))
    out["qft_x"] = np.int64(x)
    out["qft_gates"] = np.int64(len(g))
    del psi
    closed = oracle.qft_basis_amplitudes(N, x, idx)
    err = float(np.max(np.abs(amp - closed)))
    print(f"qft stride tier against the closed form: max-abs {err:.3e}", flush=True)
    if err > 1e-12:
        raise SystemExit("the oracle's two QFT results disagree; nothing written")

    np.savez(OUT + ".tmp.npz", **out)
    os.replace(OUT + ".tmp.npz", OUT)
    print(f"wrote {OUT}: {len(idx)} indices, norms {out['layers_norm']!r} / "
          f"{out['qft_norm']!r}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count() or 1)
