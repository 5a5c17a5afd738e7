/*
 * CPU reference state-vector simulator in complex128 -- TEST INFRASTRUCTURE.
 *
 * This is the oracle that the GPU library is checked against. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * GPU library never links, calls or includes it, and the two share no source.
 *
 * What it computes (R. LaRose, "Distributed Memory Techniques for Classical
 * Simulation of Quantum Circuits", arXiv:1801.01037):
 *   - the state is 2^n complex amplitudes alpha_{b_{n-1}...b_0} (State Vector
 *     Partitioning, the three-qubit binary-index equation); qubit q is bit q of
 *     the index, so a gate on qubit q pairs amplitudes 2^q apart (the stride
 *     rule and the n = 3 pairing figure of the same section);
 *   - a one-qubit gate Q = [[q11, q12], [q21, q22]] replaces every pair
 *     (a, b) = (alpha_{..0_i..}, alpha_{..1_i..}) by (q11 a + q12 b,
 *     q21 a + q22 b)  (the update equation of State Vector Partitioning);
 *   - it is applied by the two nested loops of Algorithm 1 (Single Node
 *     Implementation): an outer loop over blocks 2^{i+1} apart and an inner
 *     loop over the 2^i pairs of a block;
 *   - a gate with control c and target t runs the same update only on
 *     amplitudes whose index has bit c set (the caption of Algorithm 1);
 *   - controlled-phase is the controlled gate with Q = diag(1, e^{i theta});
 *   - a gate with several controls (the Toffoli, or controlled-controlled-NOT,
 *     gate of section Quantum Circuits is X with two) updates only where every
 *     control bit is set;
 *   - a general gate U on k qubits (q_0, ..., q_{k-1}) is the 2^k x 2^k
 *     operator of the tensor-product rule of section Quantum Information
 *     Processing acting on those qubits' factor: for every setting of the
 *     other index bits, the 2^k amplitudes a_c, c = sum_m b_{q_m} 2^m, become
 *     sum_c U[r][c] a_c (q_0 is the least significant bit of c, so U = B (x) A
 *     applies A to q_0 and B to q_1).
 *
 * Arithmetic: every complex product is written out in real arithmetic and the
 * file is built with -ffp-contract=off, so each operation rounds once.
 *
 * Threads: the reference build (liboracle.so) is single-threaded. The same
 * source built with -fopenmp (liboracle_omp.so) shares the iterations of
 * Algorithm 1's two loops, taken together, among threads (the loops of the
 * paper's Multi-Threading section). The pairs of one gate are disjoint and each
 * is updated by the same operations in the same order, so both builds give
 * the same bits; reductions (the norm) stay sequential. It serves as the all-core
 * CPU baseline and to run large reference circuits.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer iterations than this stay on one thread. */
#define ORC_PAR_MIN 4096

/* Work-sharing in the OpenMP build (nothing in the reference build):
 * ORC_FOR2 shares the iterations of Algorithm 1's two nested loops, taken
 * together, among the threads; ORC_FOR those of a single loop. Both only when
 * the flag `orc_par` in scope holds (enough work to share). */
#ifdef _OPENMP
#define ORC_FOR2 _Pragma("omp parallel for collapse(2) if(orc_par)")
#define ORC_FOR _Pragma("omp parallel for schedule(static) if(orc_par)")
#else
#define ORC_FOR2
#define ORC_FOR
#endif

#define ORC_TWO_PI 6.283185307179586476925286766559

/* Gate record as stored in the serialized gate lists (80 bytes). */
typedef struct {
    int32_t kind;     /* 0: 2x2 on target; 1: controlled 2x2; 2: controlled phase;
                         3: 2x2 with a set of controls */
    int32_t control;  /* -1 when none; kind 3: low 32 bits of the control mask */
    int32_t target;
    int32_t flags;    /* kind 3: high 32 bits of the control mask */
    double m[8];      /* q11, q12, q21, q22 as (re, im); kind 2: m[0] = theta */
} orc_gate;

enum { ORC_U = 0, ORC_CU = 1, ORC_CPHASE = 2, ORC_MCU = 3 };

/* psi is interleaved (re, im) doubles, 2^n complex entries. */

/* |x>: every amplitude 0 except alpha_x = 1 (the register starts in a basis
 * state, |0...0> in the paper's examples). */
void orc_init_basis(double *psi, int n, uint64_t x)
{
    uint64_t N = (uint64_t)1 << n;
    const int orc_par = N >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR
    for (uint64_t i = 0; i < 2 * N; ++i)
        psi[i] = 0.0;
    psi[2 * x] = 1.0;
}

/* One pair update: (a, b) <- (q11 a + q12 b, q21 a + q22 b). */
static void pair_update(double *a, double *b, const double m[8])
{
    double ar = a[0], ai = a[1], br = b[0], bi = b[1];
    double q11r = m[0], q11i = m[1], q12r = m[2], q12i = m[3];
    double q21r = m[4], q21i = m[5], q22r = m[6], q22i = m[7];
    double nar = (q11r * ar - q11i * ai) + (q12r * br - q12i * bi);
    double nai = (q11r * ai + q11i * ar) + (q12r * bi + q12i * br);
    double nbr = (q21r * ar - q21i * ai) + (q22r * br - q22i * bi);
    double nbi = (q21r * ai + q21i * ar) + (q22r * bi + q22i * br);
    a[0] = nar; a[1] = nai;
    b[0] = nbr; b[1] = nbi;
}

/* Algorithm 1: Q on qubit t. Outer loop j over blocks of 2^{t+1} amplitudes,
 * inner loop k over the first half of the block; k pairs with k + 2^t. */
void orc_apply_1q(double *psi, int n, int t, const double m[8])
{
    uint64_t N = (uint64_t)1 << n;
    uint64_t stride = (uint64_t)1 << t;
    const int orc_par = N >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR2
    for (uint64_t j = 0; j < N; j += 2 * stride)
        for (uint64_t k = j; k < j + stride; ++k)
            pair_update(psi + 2 * k, psi + 2 * (k + stride), m);
}

/* Algorithm 1 with a control qubit c: the same loops, updating only where bit
 * c of the index is one (c != t, so both members of a pair share bit c). */
void orc_apply_ctrl(double *psi, int n, int c, int t, const double m[8])
{
    uint64_t N = (uint64_t)1 << n;
    uint64_t stride = (uint64_t)1 << t;
    uint64_t cbit = (uint64_t)1 << c;
    const int orc_par = N >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR2
    for (uint64_t j = 0; j < N; j += 2 * stride)
        for (uint64_t k = j; k < j + stride; ++k)
            if (k & cbit)
                pair_update(psi + 2 * k, psi + 2 * (k + stride), m);
}

/* Algorithm 1 with a set of controls (bit mask cmask, not holding t): the
 * same loops, updating only where every control bit of the index is one. */
void orc_apply_mcu(double *psi, int n, uint64_t cmask, int t, const double m[8])
{
    uint64_t N = (uint64_t)1 << n;
    uint64_t stride = (uint64_t)1 << t;
    const int orc_par = N >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR2
    for (uint64_t j = 0; j < N; j += 2 * stride)
        for (uint64_t k = j; k < j + stride; ++k)
            if ((k & cmask) == cmask)
                pair_update(psi + 2 * k, psi + 2 * (k + stride), m);
}

/* General gate on k <= 6 distinct qubits q[0..k-1] (see the header): U is
 * 2^k x 2^k complex, row major, (re, im) interleaved. The outer loop runs over
 * the 2^(n-k) settings of the other bits (g with zeros inserted at the qubit
 * positions, in increasing order); each product is written out in real
 * arithmetic and the terms are summed in column order. Returns 0, or -1 for
 * bad arguments. */
int orc_apply_unitary(double *psi, int n, const int *q, int k, const double *U)
{
    if (k < 1 || k > 6 || k > n)
        return -1;
    int sorted[6];
    for (int m = 0; m < k; ++m) {
        if (q[m] < 0 || q[m] >= n)
            return -1;
        for (int m2 = 0; m2 < m; ++m2)
            if (q[m2] == q[m])
                return -1;
        sorted[m] = q[m];
    }
    for (int a = 1; a < k; ++a)        /* insertion sort of the positions */
        for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
            int t = sorted[b]; sorted[b] = sorted[b - 1]; sorted[b - 1] = t;
        }
    const uint64_t D = (uint64_t)1 << k;
    const uint64_t G = (uint64_t)1 << (n - k);
    uint64_t off[64];                  /* index offset of local combination c */
    for (uint64_t c = 0; c < D; ++c) {
        off[c] = 0;
        for (int m = 0; m < k; ++m)
            if ((c >> m) & 1u)
                off[c] |= (uint64_t)1 << q[m];
    }
    const int orc_par = G >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR
    for (uint64_t g = 0; g < G; ++g) {
        double a[128], out[128];
        uint64_t base = g;             /* insert a zero at each qubit position */
        for (int m = 0; m < k; ++m) {
            uint64_t low = base & (((uint64_t)1 << sorted[m]) - 1);
            base = ((base >> sorted[m]) << (sorted[m] + 1)) | low;
        }
        for (uint64_t c = 0; c < D; ++c) {
            a[2 * c] = psi[2 * (base | off[c])];
            a[2 * c + 1] = psi[2 * (base | off[c]) + 1];
        }
        for (uint64_t r = 0; r < D; ++r) {
            double re = 0.0, im = 0.0;
            for (uint64_t c = 0; c < D; ++c) {
                double ur = U[2 * (r * D + c)], ui = U[2 * (r * D + c) + 1];
                re += ur * a[2 * c] - ui * a[2 * c + 1];
                im += ur * a[2 * c + 1] + ui * a[2 * c];
            }
            out[2 * r] = re;
            out[2 * r + 1] = im;
        }
        for (uint64_t r = 0; r < D; ++r) {
            psi[2 * (base | off[r])] = out[2 * r];
            psi[2 * (base | off[r]) + 1] = out[2 * r + 1];
        }
    }
    return 0;
}

/* Controlled phase: the controlled gate with Q = diag(1, e^{i theta}). */
void orc_apply_cphase(double *psi, int n, int c, int t, double theta)
{
    double m[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, cos(theta), sin(theta)};
    orc_apply_ctrl(psi, n, c, t, m);
}

/* Threads the OpenMP build uses from now on (n >= 1); returns the number in
 * effect. The reference build always runs one thread and returns 1. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Applies the gates in list order. Returns 0, or -1 on a malformed record. */
int orc_run_circuit(double *psi, int n, const orc_gate *g, size_t count)
{
    for (size_t i = 0; i < count; ++i) {
        int t = g[i].target, c = g[i].control;
        if (t < 0 || t >= n)
            return -1;
        switch (g[i].kind) {
        case ORC_U:
            orc_apply_1q(psi, n, t, g[i].m);
            break;
        case ORC_CU:
            if (c < 0 || c >= n || c == t)
                return -1;
            orc_apply_ctrl(psi, n, c, t, g[i].m);
            break;
        case ORC_CPHASE:
            if (c < 0 || c >= n || c == t)
                return -1;
            orc_apply_cphase(psi, n, c, t, g[i].m[0]);
            break;
        case ORC_MCU: {
            uint64_t cm = (uint64_t)(uint32_t)g[i].control |
                          ((uint64_t)(uint32_t)g[i].flags << 32);
            if ((cm >> t) & 1 || (n < 64 && (cm >> n) != 0))
                return -1;
            orc_apply_mcu(psi, n, cm, t, g[i].m);
            break;
        }
        default:
            return -1;
        }
    }
    return 0;
}

/* p_i = |alpha_i|^2 for i in [first, first + count). */
void orc_probs(const double *psi, uint64_t first, uint64_t count, double *out)
{
    const int orc_par = count >= ORC_PAR_MIN;
    (void)orc_par;
    ORC_FOR
    for (uint64_t i = 0; i < count; ++i) {
        double re = psi[2 * (first + i)], im = psi[2 * (first + i) + 1];
        out[i] = re * re + im * im;
    }
}

/* Pairwise (recursive halving) sum of |alpha_i|^2 over [lo, hi). */
static double norm_range(const double *psi, uint64_t lo, uint64_t hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (uint64_t i = lo; i < hi; ++i)
            s += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        return s;
    }
    uint64_t mid = lo + (hi - lo) / 2;
    return norm_range(psi, lo, mid) + norm_range(psi, mid, hi);
}

/* sum_i |alpha_i|^2, the normalisation of the state (Quantum Information
 * Processing: the probabilities of a state sum to one). */
double orc_norm(const double *psi, int n)
{
    return norm_range(psi, 0, (uint64_t)1 << n);
}

/* Closed form of the QFT circuit (no final swaps) on the basis state |x>:
 * alpha_i = e^{2 pi i x y / 2^n} / 2^{n/2} with y = i with its n bits reversed.
 * x*y is reduced mod 2^n in 128-bit integers before it becomes an angle. */
void orc_qft_basis_amplitude(int n, uint64_t x, uint64_t i, double out[2])
{
    uint64_t y = 0;
    for (int b = 0; b < n; ++b)
        y |= ((i >> b) & 1u) << (n - 1 - b);
    unsigned __int128 prod = (unsigned __int128)x * y;
    uint64_t mask = (n == 64) ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
    uint64_t num = (uint64_t)prod & mask;
    double frac = ldexp((double)num, -n);           /* exact: num < 2^53 for n <= 53 */
    double ang = ORC_TWO_PI * frac;
    double scale = ldexp(1.0, -n / 2) * ((n & 1) ? sqrt(0.5) : 1.0);
    out[0] = cos(ang) * scale;
    out[1] = sin(ang) * scale;
}
