"""Seeded synthetic workloads: gate lists, basis states and arrival times.

This module generates *inputs* only. It holds no state-vector arithmetic: it
never applies a gate to an amplitude. Both the CPU oracle and the GPU library
consume what it produces, as plain data in one binary record format:

    struct gate {            # 80 bytes, little endian
        int32  kind;         # G_U, G_CU or G_CPHASE
        int32  control;      # control qubit, -1 when there is none
        int32  target;       # target qubit
        int32  flags;        # reserved, 0
        double m[8];         # G_U / G_CU: q11, q12, q21, q22 as (re, im) pairs,
                             # row major; G_CPHASE: m[0] = theta (radians)
    };

Qubit q is bit q of the amplitude index (stride 2^q), the convention of the
paper's stride update rule (State Vector Partitioning, the equation that pairs
amplitudes differing in the i-th index bit).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): 53-bit uniforms, normals by the
Box-Muller transform, Haar SU(2) matrices from four normals normalised onto
the 3-sphere. The paper calls its gates "random unitaries" without fixing a
distribution; Haar SU(2) is this project's reading.
"""
from __future__ import annotations

import math

import numpy as np

G_U = 0        # 2x2 unitary on `target`
G_CU = 1       # 2x2 unitary on `target`, applied where bit `control` is 1
G_CPHASE = 2   # diag(1, e^{i theta}) on `target`, controlled by `control`
G_MCU = 3      # 2x2 unitary on `target`, applied where every control bit is 1;
               # the control mask's low 32 bits are in `control`, high 32 in `flags`
G_UNITARY = 4  # 2^k x 2^k unitary on k = `control` qubits listed in 6-bit fields of
               # `flags` (first qubit lowest); `target` indexes a side table of matrices

GATE_DTYPE = np.dtype([
    ("kind", "<i4"), ("control", "<i4"), ("target", "<i4"), ("flags", "<i4"),
    ("m", "<f8", (8,)),
])
assert GATE_DTYPE.itemsize == 80

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

X_MATRIX = (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0)
_RS2 = math.sqrt(0.5)
H_MATRIX = (_RS2, 0.0, _RS2, 0.0, _RS2, 0.0, -_RS2, 0.0)


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of SplitMix64 started from state `seed`.

    Output k (k = 1, 2, ...) is mix(seed + k * golden) mod 2^64.
    """
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
    return _mix(z)


def uniform53(u64: np.ndarray) -> np.ndarray:
    """Top 53 bits as a double in [0, 1)."""
    return (u64 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def sorted_uniforms(seed: int, count: int) -> np.ndarray:
    """`count` uniforms in [0, 1) (SplitMix64, 53 bits), sorted ascending: the
    draws of a measurement sample."""
    return np.sort(uniform53(splitmix64(seed, count)))


def normals(seed: int, count: int) -> np.ndarray:
    """`count` standard normals by Box-Muller with u1 <- 1 - u1 (so u1 > 0)."""
    pairs = (count + 1) // 2
    u = uniform53(splitmix64(seed, 2 * pairs))
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * pairs)
    out[0::2] = r * np.cos(2.0 * np.pi * u2)
    out[1::2] = r * np.sin(2.0 * np.pi * u2)
    return out[:count]


def derive_seed(master: int, index: int) -> int:
    """Seed of item `index` of a family keyed by `master` (one SplitMix64 output)."""
    with np.errstate(over="ignore"):
        z = np.uint64(master & 0xFFFFFFFFFFFFFFFF) + np.uint64(index + 1) * _GOLDEN
    return int(_mix(np.array([z], dtype=np.uint64))[0])


def haar_su2(seed: int, count: int) -> np.ndarray:
    """`count` Haar-random SU(2) matrices as (count, 8) rows of gate.m.

    (a, b, c, d) uniform on S^3 gives U = [[a+ib, c+id], [-c+id, a-ib]], det 1.
    """
    g = normals(seed, 4 * count).reshape(count, 4)
    g /= np.sqrt((g * g).sum(axis=1, keepdims=True))
    a, b, c, d = g[:, 0], g[:, 1], g[:, 2], g[:, 3]
    return np.stack([a, b, c, d, -c, d, a, -b], axis=1)


def random_unitary(k: int, seed: int) -> np.ndarray:
    """A seeded Haar-random 2^k x 2^k unitary (complex128): the Q factor of a
    complex Gaussian matrix, with the phases of R's diagonal moved into Q."""
    d = 1 << k
    g = normals(seed, 2 * d * d)
    z = (g[0::2] + 1j * g[1::2]).reshape(d, d)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[np.newaxis, :]


def gate_u(target: int, m) -> np.ndarray:
    g = np.zeros(1, GATE_DTYPE)
    g["kind"], g["control"], g["target"] = G_U, -1, target
    g["m"][0] = m
    return g


def gate_cu(control: int, target: int, m) -> np.ndarray:
    g = np.zeros(1, GATE_DTYPE)
    g["kind"], g["control"], g["target"] = G_CU, control, target
    g["m"][0] = m
    return g


def gate_cnot(control: int, target: int) -> np.ndarray:
    return gate_cu(control, target, X_MATRIX)


def gate_mcu(controls, target: int, m) -> np.ndarray:
    """A 2x2 gate with a set of controls (Toffoli: gate_mcu((a, b), t, X_MATRIX))."""
    mask = 0
    for c in controls:
        mask |= 1 << int(c)
    g = np.zeros(1, GATE_DTYPE)
    g["kind"], g["target"] = G_MCU, target
    g["control"] = np.array(mask & 0xFFFFFFFF, dtype=np.uint32).view(np.int32)
    g["flags"] = np.array(mask >> 32, dtype=np.uint32).view(np.int32)
    g["m"][0] = m
    return g


def gate_unitary(qubits, index: int) -> np.ndarray:
    """A general gate on the listed qubits (k <= 5; qubits[0] is the least
    significant bit of the local index) whose matrix is entry `index` of a
    side table (see unitary_table)."""
    qs = [int(q) for q in qubits]
    if not 1 <= len(qs) <= 5:
        raise ValueError("1 to 5 qubits")
    packed = 0
    for j, q in enumerate(qs):
        packed |= q << (6 * j)
    g = np.zeros(1, GATE_DTYPE)
    g["kind"], g["control"], g["target"] = G_UNITARY, len(qs), int(index)
    g["flags"] = np.array(packed, dtype=np.uint32).view(np.int32)
    return g


def unitary_qubits(g) -> list:
    """The qubit list of a G_UNITARY record."""
    packed = int(np.array(g["flags"], dtype=np.int32).view(np.uint32))
    return [(packed >> (6 * j)) & 63 for j in range(int(g["control"]))]


def unitary_table(mats) -> np.ndarray:
    """Side table of G_UNITARY matrices: entry j holds matrix j (2^k x 2^k
    complex) in its first 2 * 4^k doubles, row major, (re, im) interleaved;
    every entry takes 2048 doubles."""
    out = np.zeros((len(mats), 2048), dtype=np.float64)
    for j, m in enumerate(mats):
        v = np.ascontiguousarray(m, dtype=np.complex128).reshape(-1).view(np.float64)
        out[j, :v.size] = v
    return out


def gate_control_mask(g) -> int:
    """The control qubits of a record as a bit mask (0 for none)."""
    kind = int(g["kind"])
    if kind == G_MCU:
        lo = int(np.array(g["control"], dtype=np.int32).view(np.uint32))
        hi = int(np.array(g["flags"], dtype=np.int32).view(np.uint32))
        return lo | (hi << 32)
    c = int(g["control"])
    return 0 if c < 0 else 1 << c


def gate_cphase(control: int, target: int, theta: float) -> np.ndarray:
    g = np.zeros(1, GATE_DTYPE)
    g["kind"], g["control"], g["target"] = G_CPHASE, control, target
    g["m"][0, 0] = theta
    return g


def layer_circuit(n: int, depth: int, seed: int) -> np.ndarray:
    """`depth` layers: a Haar SU(2) on every qubit 0..n-1 in increasing order,
    then CNOTs on neighbour pairs (control = lower qubit): pairs (0,1),(2,3),...
    in even layers and (1,2),(3,4),... in odd layers."""
    su2 = haar_su2(seed, n * depth)
    n_cnot = sum(len(range(l % 2, n - 1, 2)) for l in range(depth))
    g = np.zeros(n * depth + n_cnot, GATE_DTYPE)
    pos = 0
    for layer in range(depth):
        g["kind"][pos:pos + n] = G_U
        g["control"][pos:pos + n] = -1
        g["target"][pos:pos + n] = np.arange(n)
        g["m"][pos:pos + n] = su2[layer * n:(layer + 1) * n]
        pos += n
        for c in range(layer % 2, n - 1, 2):
            g["kind"][pos], g["control"][pos], g["target"][pos] = G_CU, c, c + 1
            g["m"][pos] = X_MATRIX
            pos += 1
    assert pos == len(g)
    return g


def qft_circuit(n: int) -> np.ndarray:
    """Quantum Fourier transform without the final swaps, n(n+1)/2 gates:
    for j = n-1 down to 0: H on j, then controlled-phase R with control m and
    target j, angle 2*pi / 2^(j-m+1), for m = j-1 down to 0."""
    g = np.zeros(n * (n + 1) // 2, GATE_DTYPE)
    pos = 0
    two_pi = 2.0 * math.pi
    for j in range(n - 1, -1, -1):
        g["kind"][pos], g["control"][pos], g["target"][pos] = G_U, -1, j
        g["m"][pos] = H_MATRIX
        pos += 1
        for m in range(j - 1, -1, -1):
            g["kind"][pos], g["control"][pos], g["target"][pos] = G_CPHASE, m, j
            g["m"][pos, 0] = two_pi / 2.0 ** (j - m + 1)
            pos += 1
    assert pos == len(g)
    return g


def inverse_circuit(gates: np.ndarray) -> np.ndarray:
    """The adjoint circuit: reversed order, each 2x2 conjugate-transposed,
    each controlled-phase angle negated (for unitary gates this undoes `gates`)."""
    inv = gates[::-1].copy()
    m = inv["m"]
    u = inv["kind"] != G_CPHASE
    q11r, q11i, q12r, q12i = m[u, 0].copy(), m[u, 1].copy(), m[u, 2].copy(), m[u, 3].copy()
    q21r, q21i, q22r, q22i = m[u, 4].copy(), m[u, 5].copy(), m[u, 6].copy(), m[u, 7].copy()
    m[u, 0], m[u, 1] = q11r, -q11i
    m[u, 2], m[u, 3] = q21r, -q21i
    m[u, 4], m[u, 5] = q12r, -q12i
    m[u, 6], m[u, 7] = q22r, -q22i
    p = ~u
    m[p, 0] = -m[p, 0]
    inv["m"] = m
    return inv


def random_basis_index(n: int, seed: int) -> int:
    """A seeded uniform basis index in [0, 2^n) (top n bits of one output)."""
    return int(splitmix64(seed, 1)[0] >> np.uint64(64 - n))


def batch_specs(master_seed: int, count: int, n_lo: int, n_hi: int,
                d_lo: int, d_hi: int):
    """(n, depth, gate_seed) for `count` circuits with n ~ U{n_lo..n_hi} and
    depth ~ U{d_lo..d_hi}, each drawn as lo + (r mod (hi - lo + 1))."""
    out = []
    for i in range(count):
        r = splitmix64(derive_seed(master_seed, i), 3)
        n = n_lo + int(r[0] % np.uint64(n_hi - n_lo + 1))
        d = d_lo + int(r[1] % np.uint64(d_hi - d_lo + 1))
        out.append((n, d, int(r[2])))
    return out


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds, from 0) of a Poisson process of `rate` per second."""
    u = uniform53(splitmix64(seed, count))
    return np.cumsum(-np.log1p(-u) / rate)


# ---- the named workloads (sizes as in the paper's single-gate benchmarks,
# ---- scaled to one GPU's memory) -------------------------------------------

def workload_layers_qft(n: int = 16, depth: int = 100, seed: int = 0) -> np.ndarray:
    """16 qubits, 100 random layers then a QFT: 1600 SU(2) + 750 CNOT + 136."""
    return np.concatenate([layer_circuit(n, depth, seed), qft_circuit(n)])


def gate_qubits(g) -> tuple:
    """Qubits a gate record touches (controls first, ascending)."""
    mask = gate_control_mask(g)
    ctrl = tuple(q for q in range(64) if (mask >> q) & 1)
    return ctrl + (int(g["target"]),)


def random_state(n: int, seed: int) -> np.ndarray:
    """A seeded normalised complex128 vector of 2^n amplitudes (i.i.d. normal
    real and imaginary parts, scaled to unit 2-norm)."""
    g = normals(seed, 2 << n)
    psi = g[0::2] + 1j * g[1::2]
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2))
