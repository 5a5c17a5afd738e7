"""The SV_FUSE_DENSE planner on the host: five-qubit blocks whose 32x32
matrices, applied in order, reproduce the circuit (checked against the
oracle's dense Kronecker tier and its stride tier). Runs without a GPU."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from oracle import dense
from tests.test_plan import mixed_circuit


def _embed(n, mask, m):
    """Full 2^n operator of a block matrix m acting on the 5 bits of mask."""
    bits = [b for b in range(n) if (mask >> b) & 1]
    others = [b for b in range(n) if not (mask >> b) & 1]
    u = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for col in range(1 << (n - 5)):
        base = sum(((col >> k) & 1) << b for k, b in enumerate(others))
        idx = [base + sum(((r >> k) & 1) << b for k, b in enumerate(bits)) for r in range(32)]
        u[np.ix_(idx, idx)] = m
    return u


@pytest.mark.parametrize("n,seed", [(5, 1), (6, 2), (7, 3), (8, 4)])
def test_blocks_reproduce_dense_tier(n, seed):
    g = mixed_circuit(n, 80, seed)
    masks, mats = sv.sv_plan_dense_inspect(n, g)
    assert all(bin(int(m)).count("1") == 5 for m in masks)
    u = np.eye(1 << n, dtype=np.complex128)
    for m, M in zip(masks, mats):
        assert np.max(np.abs(M @ M.conj().T - np.eye(32))) <= 1e-13   # unitary
        u = _embed(n, int(m), M) @ u
    ref = dense.circuit_unitary(n, g)
    assert np.max(np.abs(u - ref)) <= 1e-12


def test_blocks_reproduce_stride_tier_on_a_layer_circuit():
    n = 9
    g = qc.layer_circuit(n, 6, 3)
    masks, mats = sv.sv_plan_dense_inspect(n, g)
    psi = qc.random_state(n, 4)
    ref = psi.copy()
    oracle.run_circuit(ref, g)
    for m, M in zip(masks, mats):
        psi = _embed(n, int(m), M) @ psi
    assert np.max(np.abs(psi - ref)) <= 1e-13
    assert len(masks) < len(g) / 2          # blocks really fuse gates
