"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests touch the GPU. Each checks the oracle against something
other than itself: values the paper prints (golden fixtures), closed forms
(QFT of a basis state, H on every qubit, the product-state rule), an
independent brute-force tier (dense Kronecker operators), invariants (norm,
mirror circuits, untouched control-0 half) and brute force on tiny inputs.
"""
import math

import numpy as np
import pytest

import oracle
import qcircuits as qc
from oracle import dense
from tests.conftest import read_golden

R = math.sqrt(0.5)


def _num(tok):
    if tok == "r":
        return R
    if tok == "-r":
        return -R
    return float(tok)


def _gate_matrix(name):
    return {"X": qc.X_MATRIX, "H": qc.H_MATRIX}[name]


# ---- golden: values printed in the paper ---------------------------------

def test_pauli_x_and_hadamard_worked_values():
    for row in read_golden("pauli_x_hadamard.txt"):
        name, inp = row[0], int(row[1])
        want = np.array([complex(_num(row[2]), _num(row[3])),
                         complex(_num(row[4]), _num(row[5]))])
        psi = oracle.basis_state(1, inp)
        oracle.apply_1q(psi, 0, _gate_matrix(name))
        assert np.max(np.abs(psi - want)) <= 1e-15, (name, inp)


def test_cnot_printed_matrix_and_truth_table():
    rows = read_golden("cnot.txt")
    i = rows.index(["matrix"])
    mat = np.array([[float(v) for v in r] for r in rows[i + 1:i + 5]])
    truth = rows[rows.index(["truth"]) + 1:]
    # control = first written qubit = qubit 1, target = qubit 0
    for col in range(4):
        psi = oracle.basis_state(2, col)
        oracle.apply_ctrl(psi, 1, 0, qc.X_MATRIX)
        assert np.array_equal(psi, mat[:, col].astype(np.complex128)), col
    for src, dst in truth:
        psi = oracle.basis_state(2, int(src, 2))
        oracle.apply_ctrl(psi, 1, 0, qc.X_MATRIX)
        assert psi[int(dst, 2)] == 1.0 and np.count_nonzero(psi) == 1
    # the dense tier builds the same printed matrix
    assert np.array_equal(dense.operator_ctrl(2, 1, 0, dense.matrix_of(qc.X_MATRIX)), mat)


def _unitary_with_first_column(alpha, beta):
    # [[alpha, -conj(beta)], [beta, conj(alpha)]] maps |0> to (alpha, beta)
    a, b = complex(alpha), complex(beta)
    return (a.real, a.imag, -b.real, b.imag, b.real, b.imag, a.real, -a.imag)


def test_two_qubit_tensor_example():
    rng = np.random.default_rng(7)
    v = rng.normal(size=(2, 4))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    a0, b0 = complex(v[0, 0], v[0, 1]), complex(v[0, 2], v[0, 3])
    a1, b1 = complex(v[1, 0], v[1, 1]), complex(v[1, 2], v[1, 3])
    env = {"a0": a0, "b0": b0, "a1": a1, "b1": b1}
    psi = oracle.basis_state(2, 0)
    oracle.apply_1q(psi, 1, _unitary_with_first_column(a0, b0))   # paper's psi_0
    oracle.apply_1q(psi, 0, _unitary_with_first_column(a1, b1))   # paper's psi_1
    for idx, left, right in read_golden("tensor_2q.txt"):
        assert abs(psi[int(idx)] - env[left] * env[right]) <= 1e-15


def test_n3_pairing_strides_and_locality():
    for q, stride, where in read_golden("pairs_n3.txt"):
        q, stride = int(q), int(stride)
        psi = np.arange(8, dtype=np.complex128)
        oracle.apply_1q(psi, q, qc.X_MATRIX)
        partner = psi.real.astype(int)           # X swaps each pair
        pairs = {tuple(sorted((i, int(partner[i])))) for i in range(8)}
        assert len(pairs) == 4
        for lo, hi in pairs:
            assert hi - lo == stride
            assert ((lo < 4) == (hi < 4)) == (where == "local")


def test_qft_two_qubit_hand_values():
    for row in read_golden("qft_n2.txt"):
        x = int(row[0])
        want = np.array([complex(float(row[1 + 2 * k]), float(row[2 + 2 * k]))
                         for k in range(4)]) / 2
        psi = oracle.simulate(2, qc.qft_circuit(2), x)
        assert np.max(np.abs(psi - want)) <= 1e-15, x
        cf = oracle.qft_basis_amplitudes(2, x, range(4))
        assert np.max(np.abs(cf - want)) <= 1e-15, x


# ---- closed forms ---------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 13])
def test_qft_stride_tier_matches_closed_form(n):
    for x in {0, 1, (1 << n) - 1, qc.random_basis_index(n, 100 + n)}:
        psi = oracle.simulate(n, qc.qft_circuit(n), x)
        cf = oracle.qft_basis_amplitudes(n, x, range(1 << n))
        assert np.max(np.abs(psi - cf)) <= 1e-13, (n, x)


@pytest.mark.parametrize("n", [1, 4, 10, 18])
def test_hadamard_on_every_qubit_is_uniform(n):
    g = np.concatenate([qc.gate_u(q, qc.H_MATRIX) for q in range(n)])
    psi = oracle.simulate(n, g)
    assert np.max(np.abs(psi - oracle.uniform_amplitude(n))) <= 1e-15


def test_product_state_rule():
    n = 9
    su2 = qc.haar_su2(5, 40)
    rng = np.random.default_rng(3)
    g = np.concatenate([qc.gate_u(int(t), su2[i]) for i, t in
                        enumerate(rng.integers(0, n, size=40))])
    x = 0b101100101
    psi = oracle.simulate(n, g, x)
    vec = oracle.qubit_vectors(n, g, x)
    want = np.array([oracle.product_state_amplitude(vec, i) for i in range(1 << n)])
    # the Kronecker product of the per-qubit vectors, most significant first
    kron = np.ones(1, dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        kron = np.kron(kron, vec[q])
    assert np.max(np.abs(want - kron)) <= 1e-15
    assert np.max(np.abs(psi - want)) <= 1e-14


# ---- the brute-force tier -------------------------------------------------

def _mixed_circuit(n, count, seed):
    rng = np.random.default_rng(seed)
    su2 = qc.haar_su2(seed, count)
    out = []
    for i in range(count):
        kind = int(rng.integers(0, 3)) if n > 1 else 0
        t = int(rng.integers(0, n))
        if kind == 0:
            out.append(qc.gate_u(t, su2[i]))
            continue
        c = int(rng.integers(0, n - 1))
        c = c + 1 if c >= t else c
        if kind == 1:
            out.append(qc.gate_cu(c, t, su2[i]))
        else:
            out.append(qc.gate_cphase(c, t, float(rng.uniform(-7, 7))))
    return np.concatenate(out)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_stride_tier_matches_dense_tier(n):
    for seed in range(3):
        g = _mixed_circuit(n, 30, seed + 10 * n)
        x = seed % (1 << n)
        psi = oracle.simulate(n, g, x)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[x] = 1
        ref = dense.run_circuit(n, g, psi0)
        assert np.max(np.abs(psi - ref)) <= 1e-13, (n, seed)


def test_layer_and_qft_circuits_match_dense_tier():
    n = 6
    g = np.concatenate([qc.layer_circuit(n, 4, 9), qc.qft_circuit(n)])
    psi = oracle.simulate(n, g)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    assert np.max(np.abs(psi - dense.run_circuit(n, g, psi0))) <= 1e-13


def test_dense_operator_pins():
    n = 4
    for t in range(n):
        xop = dense.operator_1q(n, t, dense.matrix_of(qc.X_MATRIX))
        perm = np.zeros((16, 16))
        for i in range(16):
            perm[i ^ (1 << t), i] = 1
        assert np.array_equal(xop, perm)
    g = _mixed_circuit(n, 20, 4)
    u = dense.circuit_unitary(n, g)
    assert np.max(np.abs(u @ u.conj().T - np.eye(16))) <= 1e-13


# ---- invariants -----------------------------------------------------------

def test_norm_kept_and_mirror_returns_to_start():
    n = 12
    g = qc.layer_circuit(n, 10, 21)
    psi = oracle.simulate(n, g, 5)
    assert abs(oracle.norm(psi) - 1.0) <= 1e-13
    oracle.run_circuit(psi, qc.inverse_circuit(g))
    want = oracle.basis_state(n, 5)
    assert np.max(np.abs(psi - want)) <= 1e-12


def test_norm_and_probs_against_exact_sums():
    rng = np.random.default_rng(0)
    psi = (rng.normal(size=1 << 10) + 1j * rng.normal(size=1 << 10)).astype(np.complex128)
    p = oracle.probs(psi)
    assert np.array_equal(p, psi.real ** 2 + psi.imag ** 2)
    assert abs(oracle.norm(psi) - math.fsum(p)) <= 1e-12 * math.fsum(p)
    sub = oracle.probs(psi, 37, 101)
    assert np.array_equal(sub, p[37:138])
    assert oracle.probs(oracle.basis_state(5, 19))[19] == 1.0


def test_probabilities_of_circuit_results_sum_to_one():
    """A unitary circuit keeps the norm (section Quantum Information
    Processing: the squared moduli of a state's amplitudes sum to one), so
    the probabilities of its complex result must sum to 1."""
    n = 9
    psi = oracle.simulate(n, qc.workload_layers_qft(n, 6, 4))
    assert np.abs(psi.imag).max() > 0.05          # a complex state
    p = oracle.probs(psi)
    assert abs(math.fsum(p) - 1.0) <= 1e-13
    assert abs(math.fsum(oracle.probs(psi, 0, 200)) + math.fsum(oracle.probs(psi, 200))
               - 1.0) <= 1e-13


@pytest.mark.parametrize("n", [3, 8, 11])
def test_qft_probabilities_are_uniform(n):
    """The QFT of a basis state spreads it evenly: every |alpha|^2 is 2^-n
    (closed form of the transform; the amplitudes are complex, so a lost
    real or imaginary square shows)."""
    x = qc.random_basis_index(n, 31 + n)
    psi = oracle.basis_state(n, x)
    oracle.run_circuit(psi, qc.qft_circuit(n))
    p = oracle.probs(psi)
    assert np.max(np.abs(p - 2.0 ** -n)) <= 1e-15


def test_product_state_probabilities_factorise():
    """For one-qubit gates only, alpha_i is the product over qubits of each
    qubit's own amplitude (equation circuit-level), so p_i is the product of
    the per-qubit squared moduli."""
    n = 7
    g = np.concatenate([qc.gate_u(q % n, qc.haar_su2(50 + q, 1)[0]) for q in range(3 * n)])
    psi = oracle.simulate(n, g, 5)
    v = oracle.qubit_vectors(n, g, 5)
    p = oracle.probs(psi)
    for i in range(1 << n):
        want = 1.0
        for q in range(n):
            want *= abs(v[q, (i >> q) & 1]) ** 2
        assert abs(p[i] - want) <= 1e-14


def test_openmp_build_gives_the_same_bits():
    """The OpenMP build shares out the loops of each gate; every pair is
    still updated by the same operations, so its results equal the
    single-threaded build's bit for bit (gates on low and high targets take
    the outer and the inner loop sharing)."""
    n = 13
    g = np.concatenate([_mixed_circuit(n, 300, 8), qc.workload_layers_qft(n, 4, 2)])
    psi0 = qc.random_state(n, 12)
    u = qc.random_unitary(3, 4)
    outs = []
    for k in (1, 4):
        assert oracle.set_threads(k) == k
        try:
            psi = psi0.copy()
            oracle.run_circuit(psi, g)
            oracle.apply_unitary(psi, (11, 0, 6), u)
            oracle.apply_mcu(psi, (2, 12), 7, qc.haar_su2(9, 1)[0])
            outs.append((psi, oracle.probs(psi), oracle.norm(psi), oracle.basis_state(n, 77)))
        finally:
            oracle.set_threads(1)
    a, b = outs
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert np.array_equal(a[3], b[3])


def test_controlled_gate_leaves_control_zero_half_untouched():
    n, c, t = 7, 4, 1
    rng = np.random.default_rng(1)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    before = psi.copy()
    oracle.apply_ctrl(psi, c, t, qc.haar_su2(3, 1)[0])
    idx = np.arange(1 << n)
    untouched = (idx >> c) & 1 == 0
    assert np.array_equal(psi[untouched], before[untouched])
    assert not np.array_equal(psi[~untouched], before[~untouched])


def test_cphase_is_symmetric_in_control_and_target():
    n = 6
    rng = np.random.default_rng(2)
    a = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    b = a.copy()
    oracle.apply_cphase(a, 1, 4, 0.7)
    oracle.apply_cphase(b, 4, 1, 0.7)
    assert np.array_equal(a, b)


def test_malformed_gates_rejected():
    psi = oracle.basis_state(3)
    for bad in (qc.gate_u(3, qc.X_MATRIX), qc.gate_cnot(1, 1), qc.gate_cnot(-1, 0)):
        with pytest.raises(ValueError):
            oracle.run_circuit(psi, bad)


def test_toffoli_truth_table():
    """The Toffoli (controlled-controlled-NOT) gate named in section Quantum
    Circuits flips the target exactly when both controls are one; checked on
    every 3-qubit basis state for each choice of target."""
    for t in range(3):
        c = [q for q in range(3) if q != t]
        for x in range(8):
            psi = oracle.basis_state(3, x)
            oracle.apply_mcu(psi, c, t, qc.X_MATRIX)
            both = (x >> c[0]) & 1 and (x >> c[1]) & 1
            y = x ^ (1 << t) if both else x
            assert psi[y] == 1.0 and np.count_nonzero(psi) == 1, (t, x)


@pytest.mark.parametrize("controls,t", [((0,), 3), ((5, 1), 0), ((0, 2, 4), 5), ((1, 2, 3, 4), 0),
                                        ((0, 1, 2, 3, 4), 5)])
def test_mcu_stride_tier_matches_dense_tier(controls, t):
    n = 6
    u = qc.haar_su2(77 + t, 1)[0]
    psi = qc.random_state(n, 31 + len(controls))
    ref = dense.operator_mcu(n, controls, t, dense.matrix_of(u)) @ psi
    got = psi.copy()
    oracle.apply_mcu(got, controls, t, u)
    assert np.max(np.abs(got - ref)) < 1e-14
    # the gate record runs the same update through the circuit entry point
    got2 = psi.copy()
    oracle.run_circuit(got2, qc.gate_mcu(controls, t, u))
    assert np.array_equal(got2, got)


# ---- general gates on k qubits -----------------------------------------------

def test_unitary_on_one_qubit_is_the_stride_update():
    """k = 1 is the paper's pair update itself, bit for bit."""
    n = 7
    m = qc.haar_su2(5, 1)[0]
    u = dense.matrix_of(m)
    for t in (0, 3, 6):
        psi = qc.random_state(n, 40 + t)
        a, b = psi.copy(), psi.copy()
        oracle.apply_1q(a, t, m)
        oracle.apply_unitary(b, (t,), u)
        assert np.array_equal(a, b)


def test_unitary_tensor_product_of_one_qubit_gates():
    """U = B (x) A on (q0, q1) is A on q0 and B on q1 (tensor-product rule;
    q0 is the low bit of the local index), for both qubit orders."""
    n = 6
    ma, mb = qc.haar_su2(9, 2)
    A, B = dense.matrix_of(ma), dense.matrix_of(mb)
    for q0, q1 in ((1, 4), (4, 1), (0, 5), (3, 2)):
        psi = qc.random_state(n, 7 * q0 + q1)
        ref = psi.copy()
        oracle.apply_1q(ref, q0, ma)
        oracle.apply_1q(ref, q1, mb)
        got = psi.copy()
        oracle.apply_unitary(got, (q0, q1), np.kron(B, A))
        assert np.max(np.abs(got - ref)) < 1e-15, (q0, q1)


def test_unitary_cnot_matrix_is_the_controlled_x():
    """The 4x4 CNOT (control q0, target q1; local index b_q0 + 2 b_q1) equals
    the controlled gate of Algorithm 1's caption with Q = X."""
    cnot = np.zeros((4, 4))
    cnot[0, 0] = cnot[2, 2] = cnot[3, 1] = cnot[1, 3] = 1.0
    n = 5
    for c, t in ((0, 3), (4, 1), (2, 3)):
        psi = qc.random_state(n, 10 * c + t)
        ref = psi.copy()
        oracle.apply_ctrl(ref, c, t, qc.X_MATRIX)
        got = psi.copy()
        oracle.apply_unitary(got, (c, t), cnot)
        assert np.array_equal(got, ref), (c, t)


@pytest.mark.parametrize("qubits", [(2,), (0, 6), (5, 1), (3, 0, 6), (6, 2, 4, 1), (1, 5, 0, 3, 4)])
def test_unitary_stride_tier_matches_dense_tier(qubits):
    n = 7
    u = qc.random_unitary(len(qubits), 100 + sum(qubits))
    psi = qc.random_state(n, 55 + len(qubits))
    ref = dense.operator_unitary(n, qubits, u) @ psi
    got = psi.copy()
    oracle.apply_unitary(got, qubits, u)
    assert np.max(np.abs(got - ref)) < 1e-14
    assert abs(oracle.norm(got) - 1.0) < 1e-13   # a unitary keeps the norm


def test_unitary_qubit_order_permutes_the_matrix():
    """Listing the qubits in another order is the same gate with its local
    index bits permuted: U on (a, b) equals P U P on (b, a), P the swap of the
    two local bits."""
    n = 6
    u = qc.random_unitary(2, 3)
    P = np.eye(4)[[0, 2, 1, 3]]
    psi = qc.random_state(n, 8)
    a, b = psi.copy(), psi.copy()
    oracle.apply_unitary(a, (1, 4), u)
    oracle.apply_unitary(b, (4, 1), P @ u @ P)
    assert np.max(np.abs(a - b)) < 1e-15


def test_unitary_rejects_bad_qubits():
    psi = qc.random_state(4, 1)
    for q in ((1, 1), (4,), (-1,), (0, 1, 2, 3, 0)):
        with pytest.raises(ValueError):
            oracle.apply_unitary(psi, q, np.eye(1 << len(q)))


def test_sampling_of_a_basis_state_and_of_the_uniform_state():
    """Measurement (section Quantum Circuits) of |x> always gives x; of the
    uniform state (H on every qubit, even n: every probability exactly 2^-n,
    so every CDF value is exact) the draw u gives floor(u 2^n) exactly."""
    u = qc.sorted_uniforms(5, 4000)
    for n, x in ((1, 1), (6, 37), (10, 1000)):
        assert (oracle.sample_indices(oracle.basis_state(n, x), u) == x).all()
    for n in (2, 8, 12):
        psi = np.full(1 << n, oracle.uniform_amplitude(n), dtype=np.complex128)
        want = np.floor(u * 2.0 ** n).astype(np.uint64)
        assert np.array_equal(oracle.sample_indices(psi, u), want), n


def test_sampling_frequencies_follow_the_probabilities():
    """Chi-square of 200k draws from a seeded 8-qubit state against |alpha|^2:
    a dropped square or a shifted index fails it."""
    n = 8
    psi = qc.random_state(n, 808)
    p = np.abs(psi) ** 2
    u = qc.sorted_uniforms(9, 200000)
    counts = np.bincount(oracle.sample_indices(psi, u).astype(np.int64), minlength=1 << n)
    exp = p * len(u)
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 255 degrees of freedom: mean 255, sd ~22.6; a wrong distribution gives thousands
    assert chi2 < 400, chi2
    # zero-probability indices are never drawn, and draws near 1 take the last non-zero index
    psi2 = np.zeros(16, dtype=np.complex128)
    psi2[[2, 5, 9]] = [0.6, 0.0, 0.8]
    got = oracle.sample_indices(psi2, np.array([0.0, 0.35, 0.37, 0.999999, np.nextafter(1.0, 0.0)]))
    assert list(got) == [2, 2, 9, 9, 9]


def test_general_gate_records_follow_the_dense_tier():
    """Records of general gates (kind 4, matrices from a side table) are
    applied in list order among the other records: the stride tier equals
    the dense Kronecker tier on a circuit where they do not commute with
    their neighbours."""
    from oracle import dense
    n = 7
    mats = [qc.random_unitary(k, 20 + k) for k in (2, 3, 5, 1)]
    tab = qc.unitary_table(mats)
    g = np.concatenate([qc.layer_circuit(n, 2, 1), qc.gate_unitary([3, 0], 0),
                        qc.layer_circuit(n, 1, 2), qc.gate_unitary([6, 2, 4], 1),
                        qc.gate_unitary([1, 5, 0, 6, 3], 2), qc.gate_unitary([4], 3),
                        qc.gate_cnot(4, 5), qc.gate_unitary([5, 4], 0)])
    psi0 = qc.random_state(n, 8)
    a = psi0.copy()
    oracle.run_circuit(a, g, tab)
    b = dense.run_circuit(n, g, psi0, tab)
    assert np.max(np.abs(a - b)) <= 1e-13
    # the same gates in another order give another state
    c = psi0.copy()
    oracle.run_circuit(c, g[::-1].copy(), tab)
    assert np.max(np.abs(a - c)) > 1e-3
