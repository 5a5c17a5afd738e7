"""The seeded workload generators: determinism, counts and published vectors."""
import numpy as np

import qcircuits as qc
from oracle import dense


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 from state 0, as given by its published
    # reference implementation
    out = qc.splitmix64(0, 3)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                     0x06C45D188009454F]


def test_uniform_and_normals_are_sane():
    u = qc.uniform53(qc.splitmix64(11, 100000))
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
    g = qc.normals(12, 100001)
    assert len(g) == 100001 and abs(g.mean()) < 0.02 and abs(g.std() - 1) < 0.02


def test_haar_su2_is_special_unitary():
    m = qc.haar_su2(1, 500)
    for row in m[:50]:
        u = dense.matrix_of(row)
        assert np.allclose(u @ u.conj().T, np.eye(2), atol=1e-15)
        assert abs(np.linalg.det(u) - 1) < 1e-15


def test_gate_counts_of_the_workloads():
    assert len(qc.workload_layers_qft(16, 100, 0)) == 1600 + 750 + 136
    g = qc.layer_circuit(30, 20, 1)
    assert (g["kind"] == qc.G_U).sum() == 600 and (g["kind"] == qc.G_CU).sum() == 290
    assert len(qc.layer_circuit(33, 10, 2)) == 490
    assert len(qc.layer_circuit(34, 10, 2)) == 505
    assert len(qc.qft_circuit(30)) == 465


def test_layer_structure():
    g = qc.layer_circuit(5, 2, 3)
    assert list(g["target"][:5]) == [0, 1, 2, 3, 4]
    assert [(c, t) for c, t in zip(g["control"][5:7], g["target"][5:7])] == [(0, 1), (2, 3)]
    assert [(c, t) for c, t in zip(g["control"][12:], g["target"][12:])] == [(1, 2), (3, 4)]


def test_generators_are_deterministic():
    a = qc.layer_circuit(8, 5, 42)
    b = qc.layer_circuit(8, 5, 42)
    assert a.tobytes() == b.tobytes()
    assert qc.layer_circuit(8, 5, 43).tobytes() != a.tobytes()
    assert qc.batch_specs(7, 20, 10, 24, 20, 200) == qc.batch_specs(7, 20, 10, 24, 20, 200)


def test_batch_specs_ranges():
    specs = qc.batch_specs(0, 512, 10, 24, 20, 200)
    ns = [s[0] for s in specs]
    ds = [s[1] for s in specs]
    assert min(ns) == 10 and max(ns) == 24
    assert 20 <= min(ds) and max(ds) <= 200


def test_inverse_circuit_is_adjoint():
    n = 3
    g = np.concatenate([qc.layer_circuit(n, 2, 5), qc.qft_circuit(n)])
    u = dense.circuit_unitary(n, g)
    v = dense.circuit_unitary(n, qc.inverse_circuit(g))
    assert np.allclose(v @ u, np.eye(8), atol=1e-14)


def test_poisson_arrivals():
    t = qc.poisson_arrivals(100.0, 20000, 1)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 0.01) < 0.0005
