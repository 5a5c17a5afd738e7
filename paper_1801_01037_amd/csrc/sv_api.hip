// The C ABI declared in include/sv.h: argument checks, handle management and
// dispatch of each request to the kernels. No exception leaves this file.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "sv_internal.h"
#include "plan.h"

namespace {

thread_local std::string g_err;

sv_status fail(sv_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sv_status hip_fail(hipError_t e, const char *what)
{
    return fail(SV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SV_HIP(call, what)                            \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Makes the handle's device current for the scope of one call.
class DeviceScope {
public:
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev_) == hipSuccess && prev_ != dev && hipSetDevice(dev) == hipSuccess)
            switched_ = true;
    }
    ~DeviceScope()
    {
        if (switched_) (void)hipSetDevice(prev_);
    }

private:
    int prev_ = 0;
    bool switched_ = false;
};

bool valid_dtype(sv_dtype dt) { return dt == SV_C64 || dt == SV_C128; }

uint64_t state_bytes(const sv_state_s *s) { return (uint64_t(1) << s->n) * svk::elem_bytes(s->dt); }

sv_status check_handle(sv_state s)
{
    if (!s) return fail(SV_EINVAL, "null state handle");
    return SV_OK;
}

sv_status make_handle(void *psi, int n, sv_dtype dt, void *stream, bool owned, sv_state *out)
{
    sv_state_s *s = new (std::nothrow) sv_state_s;
    if (!s) return fail(SV_ENOMEM, "host allocation of the handle failed");
    s->psi = psi;
    s->n = n;
    s->dt = dt;
    s->stream = static_cast<hipStream_t>(stream);
    s->owned = owned;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    hipError_t e = hipMalloc(&s->scratch, (svk::kNormBlocks + 1) * sizeof(double));
    if (e != hipSuccess) {
        delete s;
        return fail(SV_ENOMEM, "hipMalloc of reduction scratch failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return SV_OK;
}

// The control qubits of a (validated) gate record as a bit mask.
uint64_t control_mask(const sv_gate &g)
{
    if (g.kind == SV_G_MCU)
        return uint64_t(uint32_t(g.control)) | (uint64_t(uint32_t(g.flags)) << 32);
    return g.kind == SV_G_U ? 0 : uint64_t(1) << g.control;
}

// Dense blocks span at most five qubits: a gate with several controls that
// touches more runs as its own launch between dense segments.
bool outside_dense_blocks(const sv_gate &g)
{
    return g.kind == SV_G_MCU && __builtin_popcountll(control_mask(g)) + 1 > 5;
}

// Dense plans (host-only inspection) hold gates of at most five qubits.
sv_status reject_wide(const sv_gate *gates, size_t n_gates)
{
    for (size_t i = 0; i < n_gates; ++i)
        if (outside_dense_blocks(gates[i]))
            return fail(SV_EUNSUPPORTED, "gate %zu: more than five qubits do not fit a dense block", i);
    return SV_OK;
}

// Queues one gate as its own kernel (one pass over the touched amplitudes).
sv_status queue_gate(sv_state s, const sv_gate &g)
{
    svk::Mat2 m;
    std::memcpy(m.q, g.m, sizeof m.q);
    const double N = std::ldexp(1.0, s->n), sb = svk::elem_bytes(s->dt);
    const uint64_t tbit = uint64_t(1) << g.target;
    const uint64_t cm = control_mask(g);
    const uint64_t both = tbit | cm;
    const bool ctrl = cm != 0;
    // Kind of kernel, and the amplitudes it must read and write.
    enum { PAIR, SWAP, DIAG } how;
    if (g.kind == SV_G_CPHASE) how = DIAG;
    else if (svk::is_pauli_x(g.m)) how = SWAP;
    else if (svk::is_phase_diag(g.m)) how = DIAG;
    else how = PAIR;
    // Amplitudes whose 128-byte lines the kernel must read and write: only a
    // control (or, for a phase, the target) on a bit that selects whole lines
    // (bit >= 3 for complex128, >= 4 for complex64) halves the lines touched.
    const int line_bit = s->dt == SV_C64 ? 4 : 3;
    const uint64_t line_sel = ~((uint64_t(1) << line_bit) - 1);
    const int nsel = __builtin_popcountll(cm & line_sel) +
                     ((how == DIAG && (tbit & line_sel)) ? 1 : 0);
    const double touched = std::ldexp(N, -nsel);
    int cls;
    double flops;
    if (how == PAIR) { cls = ctrl ? svk::KC_PAIR_CTRL : svk::KC_PAIR; flops = 14 * touched; }
    else if (how == SWAP) { cls = svk::KC_SWAP; flops = 0; }
    else { cls = svk::KC_DIAG; flops = 6 * touched; }

    const int tok = svk::prof_begin(s);
    hipError_t e;
    if (how == PAIR || how == SWAP) {
        e = svk::launch_pair(s->psi, s->n, s->dt, g.target, cm, m, how == SWAP, s->stream);
    } else {
        const double theta = g.kind == SV_G_CPHASE ? g.m[0] : std::atan2(g.m[7], g.m[6]);
        svk::DiagTerm t{both, both, svk::angle_to_turn(theta)};
        e = svk::launch_diag(s->psi, s->n, s->dt, &t, 1, s->stream);
    }
    svk::prof_end(s, tok, cls, 2 * touched * sb, flops);
    if (e != hipSuccess) return hip_fail(e, "gate kernel launch");
    return SV_OK;
}

// The qubits of a SV_G_UNITARY record (q[0] first); returns k, or 0 when the
// list is malformed for an n-qubit register.
int unitary_qubits(const sv_gate &g, int n, int32_t q[5])
{
    const int k = g.control;
    if (k < 1 || k > 5 || k > n) return 0;
    if (k < 5 && (uint32_t(g.flags) >> (6 * k)) != 0) return 0;   // stray bits past the list
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        q[j] = (uint32_t(g.flags) >> (6 * j)) & 63u;
        if (q[j] >= n || ((seen >> q[j]) & 1)) return 0;
        seen |= uint64_t(1) << q[j];
    }
    return k;
}

sv_status validate_gate(const sv_state_s *s, const sv_gate &g, size_t idx, size_t n_mats = 0)
{
    if (g.kind == SV_G_UNITARY) {
        int32_t q[5];
        if (!n_mats)
            return fail(SV_EINVAL, "gate %zu: SV_G_UNITARY records need the matrix table of "
                        "sv_run_circuit_ex", idx);
        if (!unitary_qubits(g, s->n, q))
            return fail(SV_EINVAL, "gate %zu: malformed qubit list of a SV_G_UNITARY record", idx);
        if (g.target < 0 || size_t(g.target) >= n_mats)
            return fail(SV_EINVAL, "gate %zu: matrix index %d not below %zu", idx, g.target, n_mats);
        return SV_OK;
    }
    if (g.flags != 0 && g.kind != SV_G_MCU) return fail(SV_EINVAL, "gate %zu: flags must be 0", idx);
    if (g.target < 0 || g.target >= s->n)
        return fail(SV_EINVAL, "gate %zu: target %d out of range [0, %d)", idx, g.target, s->n);
    switch (g.kind) {
    case SV_G_U:
        if (g.control != -1) return fail(SV_EINVAL, "gate %zu: SV_G_U takes control -1", idx);
        break;
    case SV_G_CU:
    case SV_G_CPHASE:
        if (g.control < 0 || g.control >= s->n)
            return fail(SV_EINVAL, "gate %zu: control %d out of range [0, %d)", idx, g.control, s->n);
        if (g.control == g.target)
            return fail(SV_EINVAL, "gate %zu: control equals target (%d)", idx, g.target);
        break;
    case SV_G_MCU: {
        const uint64_t cm = control_mask(g);
        if (cm == 0) return fail(SV_EINVAL, "gate %zu: SV_G_MCU needs at least one control", idx);
        if (s->n < 64 && (cm >> s->n) != 0)
            return fail(SV_EINVAL, "gate %zu: control mask has a bit at or above n = %d", idx, s->n);
        if ((cm >> g.target) & 1)
            return fail(SV_EINVAL, "gate %zu: control mask holds the target (%d)", idx, g.target);
        break;
    }
    default:
        return fail(SV_EINVAL, "gate %zu: unknown kind %d", idx, g.kind);
    }
    const int nm = g.kind == SV_G_CPHASE ? 1 : 8;
    for (int k = 0; k < nm; ++k)
        if (!std::isfinite(g.m[k])) return fail(SV_EINVAL, "gate %zu: non-finite matrix entry", idx);
    return SV_OK;
}

}  // namespace

namespace svk {

sv_status queue_gate(sv_state s, const sv_gate &g) { return ::queue_gate(s, g); }

sv_status set_error(sv_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

uint64_t angle_to_turn(double theta)
{
    // theta / (2 pi) as a fraction of a turn in [0, 1), scaled by 2^64. For
    // theta = (2 pi) / 2^k the quotient is exactly 2^-k.
    const double two_pi = 6.283185307179586476925286766559;
    double f = theta / two_pi;
    f -= std::floor(f);
    double scaled = std::ldexp(f, 64);
    if (!(scaled < 18446744073709551616.0)) return 0;
    return uint64_t(scaled);
}

bool is_pauli_x(const double m[8])
{
    return m[0] == 0 && m[1] == 0 && m[2] == 1 && m[3] == 0 && m[4] == 1 && m[5] == 0 &&
           m[6] == 0 && m[7] == 0;
}

bool is_phase_diag(const double m[8])
{
    if (!(m[0] == 1 && m[1] == 0 && m[2] == 0 && m[3] == 0 && m[4] == 0 && m[5] == 0))
        return false;
    const double mod2 = m[6] * m[6] + m[7] * m[7];
    return std::fabs(mod2 - 1.0) <= 4e-16;
}

}  // namespace svk

extern "C" {

int sv_version(void) { return 3; }

const char *sv_last_error(void) { return g_err.c_str(); }

sv_status sv_create(int n_qubits, sv_dtype dtype, void *hip_stream, sv_state *out)
{
    if (!out) return fail(SV_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (!valid_dtype(dtype)) return fail(SV_EINVAL, "unknown dtype %d", int(dtype));
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d not in [1, 34]", n_qubits);
    const uint64_t bytes = (uint64_t(1) << n_qubits) * svk::elem_bytes(dtype);
    void *psi = nullptr;
    hipError_t e = hipMalloc(&psi, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "hipMalloc of %llu bytes failed: %s", (unsigned long long)bytes,
                    hipGetErrorString(e));
    }
    sv_state s = nullptr;
    sv_status st = make_handle(psi, n_qubits, dtype, hip_stream, true, &s);
    if (st != SV_OK) {
        (void)hipFree(psi);
        return st;
    }
    e = svk::launch_init(psi, n_qubits, dtype, 0, s->stream);
    if (e != hipSuccess) {
        sv_destroy(s);
        return hip_fail(e, "init kernel launch");
    }
    *out = s;
    return SV_OK;
}

sv_status sv_wrap(void *dev_ptr, int n_qubits, sv_dtype dtype, void *hip_stream, sv_state *out)
{
    if (!out) return fail(SV_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (!dev_ptr) return fail(SV_EINVAL, "null device pointer");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 16 != 0)
        return fail(SV_EINVAL, "device pointer is not 16-byte aligned");
    if (!valid_dtype(dtype)) return fail(SV_EINVAL, "unknown dtype %d", int(dtype));
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d not in [1, 34]", n_qubits);
    return make_handle(dev_ptr, n_qubits, dtype, hip_stream, false, out);
}

sv_status sv_destroy(sv_state s)
{
    if (!s) return SV_OK;
    DeviceScope ds(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    svk::circuit_graph_release(s);
    svk::plan_release(s);
    svk::prof_release(s);
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->sample_scratch) (void)hipFree(s->sample_scratch);
    if (s->owned && s->psi) (void)hipFree(s->psi);
    delete s;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize in sv_destroy");
    return SV_OK;
}

sv_status sv_set_stream(sv_state s, void *hip_stream)
{
    if (sv_status st = check_handle(s)) return st;
    s->stream = static_cast<hipStream_t>(hip_stream);
    return SV_OK;
}

sv_status sv_set_tile_geometry(sv_state s, int32_t tile_qubits, int32_t register_qubits,
                               int32_t low_qubits)
{
    if (sv_status st = check_handle(s)) return st;
    if (tile_qubits != 0 && (tile_qubits < 4 || tile_qubits > svk::kTileL128))
        return fail(SV_EINVAL, "tile_qubits must be 0 (default) or 4..12");
    if (register_qubits != 0 && register_qubits != 3 && register_qubits != 4)
        return fail(SV_EINVAL, "register_qubits must be 0 (default), 3 or 4");
    if (low_qubits < -1 || low_qubits > 11)
        return fail(SV_EINVAL, "low_qubits must be -1 (default) or 0..11");
    // A captured circuit graph holds launches planned with the old geometry.
    svk::circuit_graph_release(s);
    s->tile_L = tile_qubits;
    s->tile_K = register_qubits;
    s->tile_nlow = low_qubits;
    return SV_OK;
}

sv_status sv_info(sv_state s, void **dev_ptr, int *n_qubits, sv_dtype *dtype)
{
    if (sv_status st = check_handle(s)) return st;
    if (dev_ptr) *dev_ptr = s->psi;
    if (n_qubits) *n_qubits = s->n;
    if (dtype) *dtype = s->dt;
    return SV_OK;
}

sv_status sv_reset(sv_state s, uint64_t basis_index)
{
    if (sv_status st = check_handle(s)) return st;
    if (basis_index >> s->n)
        return fail(SV_EINVAL, "basis index %llu >= 2^%d", (unsigned long long)basis_index, s->n);
    DeviceScope ds(s->device);
    const int tok = svk::prof_begin(s);
    hipError_t e = svk::launch_init(s->psi, s->n, s->dt, basis_index, s->stream);
    svk::prof_end(s, tok, svk::KC_INIT, double(state_bytes(s)), 0);
    if (e != hipSuccess) return hip_fail(e, "init kernel launch");
    return SV_OK;
}

sv_status sv_reset_uniform(sv_state s)
{
    if (sv_status st = check_handle(s)) return st;
    DeviceScope ds(s->device);
    // 2^{-n/2}: exact for even n, one rounding of 1/sqrt(2) otherwise
    const double amp = std::ldexp(s->n % 2 ? std::sqrt(0.5) : 1.0, -(s->n / 2));
    const int tok = svk::prof_begin(s);
    hipError_t e = svk::launch_fill(s->psi, s->n, s->dt, amp, s->stream);
    svk::prof_end(s, tok, svk::KC_INIT, double(state_bytes(s)), 0);
    if (e != hipSuccess) return hip_fail(e, "uniform init kernel launch");
    return SV_OK;
}

sv_status sv_apply_1q(sv_state s, int target, const double m[8])
{
    if (sv_status st = check_handle(s)) return st;
    if (!m) return fail(SV_EINVAL, "null matrix");
    sv_gate g{SV_G_U, -1, target, 0, {}};
    std::memcpy(g.m, m, sizeof g.m);
    if (sv_status st = validate_gate(s, g, 0)) return st;
    DeviceScope ds(s->device);
    return queue_gate(s, g);
}

sv_status sv_apply_ctrl(sv_state s, int control, int target, const double m[8])
{
    if (sv_status st = check_handle(s)) return st;
    if (!m) return fail(SV_EINVAL, "null matrix");
    sv_gate g{SV_G_CU, control, target, 0, {}};
    std::memcpy(g.m, m, sizeof g.m);
    if (sv_status st = validate_gate(s, g, 0)) return st;
    DeviceScope ds(s->device);
    return queue_gate(s, g);
}

sv_status sv_apply_mcu(sv_state s, uint64_t control_mask, int target, const double m[8])
{
    if (sv_status st = check_handle(s)) return st;
    if (!m) return fail(SV_EINVAL, "null matrix");
    sv_gate g{SV_G_MCU, int32_t(uint32_t(control_mask)), target,
              int32_t(uint32_t(control_mask >> 32)), {}};
    std::memcpy(g.m, m, sizeof g.m);
    if (sv_status st = validate_gate(s, g, 0)) return st;
    DeviceScope ds(s->device);
    return queue_gate(s, g);
}

sv_status sv_apply_unitary(sv_state s, const int32_t *qubits, int32_t k, const double *u)
{
    if (sv_status st = check_handle(s)) return st;
    if (!qubits || !u) return fail(SV_EINVAL, "null qubit list or matrix");
    if (k < 1 || k > 5 || k > s->n) return fail(SV_EINVAL, "k = %d not in [1, min(5, n)]", k);
    uint64_t seen = 0;
    for (int m = 0; m < k; ++m) {
        if (qubits[m] < 0 || qubits[m] >= s->n)
            return fail(SV_EINVAL, "qubit %d out of range [0, %d)", qubits[m], s->n);
        if ((seen >> qubits[m]) & 1) return fail(SV_EINVAL, "qubit %d listed twice", qubits[m]);
        seen |= uint64_t(1) << qubits[m];
    }
    DeviceScope ds(s->device);
    if (k == 1) {   // the pair update itself
        sv_gate g{SV_G_U, -1, qubits[0], 0, {}};
        std::memcpy(g.m, u, sizeof g.m);
        return queue_gate(s, g);
    }
    std::string err;
    sv_status st = svk::apply_unitary(s, qubits, k, u, &err);
    if (st != SV_OK) return fail(st, "%s", err.c_str());
    return SV_OK;
}

sv_status sv_apply_cphase(sv_state s, int control, int target, double theta)
{
    if (sv_status st = check_handle(s)) return st;
    sv_gate g{SV_G_CPHASE, control, target, 0, {theta}};
    if (sv_status st = validate_gate(s, g, 0)) return st;
    DeviceScope ds(s->device);
    return queue_gate(s, g);
}

sv_status sv_run_circuit(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags)
{
    return sv_run_circuit_ex(s, gates, n_gates, nullptr, 0, flags);
}

sv_status sv_run_circuit_ex(sv_state s, const sv_gate *gates, size_t n_gates, const double *mats,
                            size_t n_mats, uint32_t flags)
{
    if (sv_status st = check_handle(s)) return st;
    if (n_gates == 0) return SV_OK;
    if (!gates) return fail(SV_EINVAL, "null gate array");
    if (n_mats && !mats) return fail(SV_EINVAL, "null matrix table");
    if (flags & ~(SV_FUSE | SV_FUSE_DENSE | SV_GRAPH | SV_NO_RELABEL | SV_JIT))
        return fail(SV_EINVAL, "unknown flags 0x%x", flags);
    if ((flags & SV_NO_RELABEL) && !(flags & SV_FUSE))
        return fail(SV_EINVAL, "SV_NO_RELABEL applies to SV_FUSE only");
    if ((flags & SV_JIT) && !(flags & SV_FUSE))
        return fail(SV_EINVAL, "SV_JIT applies to SV_FUSE only");
    if ((flags & SV_FUSE) && (flags & SV_FUSE_DENSE))
        return fail(SV_EINVAL, "SV_FUSE and SV_FUSE_DENSE are exclusive");
    bool any_unitary = false;
    for (size_t i = 0; i < n_gates; ++i) {
        if (sv_status st = validate_gate(s, gates[i], i, n_mats)) return st;
        any_unitary |= gates[i].kind == SV_G_UNITARY;
    }
    if (any_unitary)
        for (size_t i = 0; i < n_gates; ++i)
            if (gates[i].kind == SV_G_UNITARY)
                for (int v = 0; v < 2 * (1 << (2 * gates[i].control)); ++v)
                    if (!std::isfinite(mats[size_t(gates[i].target) * 2048 + size_t(v)]))
                        return fail(SV_EINVAL, "gate %zu: non-finite matrix entry", i);
    DeviceScope ds(s->device);
    // A general gate: one launch, as sv_apply_unitary queues it.
    auto unitary = [&](const sv_gate &g) -> sv_status {
        int32_t q[5];
        const int k = unitary_qubits(g, s->n, q);
        const double *u = mats + size_t(g.target) * 2048;
        if (k == 1) {
            sv_gate one{SV_G_U, -1, q[0], 0, {}};
            std::memcpy(one.m, u, sizeof one.m);
            return queue_gate(s, one);
        }
        std::string err;
        sv_status st = svk::apply_unitary(s, q, k, u, &err);
        return st == SV_OK ? SV_OK : fail(st, "%s", err.c_str());
    };
    if (flags & SV_GRAPH) {
        if (any_unitary)
            return fail(SV_EUNSUPPORTED, "SV_GRAPH takes no SV_G_UNITARY records");
        std::string err;
        sv_status st = svk::circuit_graph_run(s, gates, n_gates, flags, &err);
        if (st != SV_OK) return fail(st, "%s", err.c_str());
        return SV_OK;
    }
    if (flags & (SV_FUSE | SV_FUSE_DENSE)) {
        // Dense blocks hold at most five qubits: wider gates with several
        // controls run as their own launches between the planned segments of
        // the other gates (list order is kept), and so do general gates.
        const bool dense = (flags & SV_FUSE_DENSE) && s->n >= 9;
        auto alone = [&](const sv_gate &g) {
            return g.kind == SV_G_UNITARY || (dense && outside_dense_blocks(g));
        };
        size_t i = 0;
        while (i < n_gates) {
            if (alone(gates[i])) {
                sv_status st = gates[i].kind == SV_G_UNITARY ? unitary(gates[i]) : queue_gate(s, gates[i]);
                if (st != SV_OK) return st;
                ++i;
                continue;
            }
            size_t j = i;
            while (j < n_gates && !alone(gates[j])) ++j;
            std::string err;
            sv_status st = svk::plan_run(s, gates + i, j - i, flags, &err);
            if (st != SV_OK) return fail(st, "%s", err.c_str());
            i = j;
        }
        return SV_OK;
    }
    for (size_t i = 0; i < n_gates; ++i) {
        sv_status st = gates[i].kind == SV_G_UNITARY ? unitary(gates[i]) : queue_gate(s, gates[i]);
        if (st != SV_OK) return st;
    }
    return SV_OK;
}

sv_status sv_run_batch(sv_state *states, const sv_gate *const *circuits, const size_t *lens,
                       size_t count, uint32_t flags)
{
    if (count == 0) return SV_OK;
    if (!states || !circuits || !lens) return fail(SV_EINVAL, "null argument array");
    if (flags & ~(SV_FUSE | SV_GRAPH)) return fail(SV_EINVAL, "unknown batch flags 0x%x", flags);
    // Everything is checked before anything runs, so an invalid argument
    // leaves every state untouched.
    std::vector<sv_state> sorted(states, states + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(SV_EINVAL, "a state appears twice in the batch");
    for (size_t c = 0; c < count; ++c) {
        if (sv_status st = check_handle(states[c])) return st;
        if (lens[c] && !circuits[c]) return fail(SV_EINVAL, "null gate array for circuit %zu", c);
        for (size_t i = 0; i < lens[c]; ++i)
            if (sv_status st = validate_gate(states[c], circuits[c][i], i)) return st;
    }
    // Circuits the planner takes (n >= 4) go into one batch per dtype; the
    // others run alone, planned, on their own streams.
    std::vector<sv_plan> plans[2];
    std::vector<sv_state> owners[2];
    std::vector<size_t> alone;
    auto destroy_plans = [&]() {
        for (auto &v : plans)
            for (sv_plan p : v) sv_plan_destroy(p);
    };
    for (size_t c = 0; c < count; ++c) {
        const sv_gate *g = circuits[c];
        if (lens[c] == 0) continue;
        if (states[c]->n < 4) {
            alone.push_back(c);
            continue;
        }
        sv_plan p = nullptr;
        if (sv_status st = sv_plan_create(states[c], g, lens[c], &p)) {
            destroy_plans();
            return st;
        }
        const int d = states[c]->dt == SV_C64 ? 0 : 1;
        plans[d].push_back(p);
        owners[d].push_back(states[c]);
    }
    sv_status result = SV_OK;
    for (int d = 0; d < 2 && result == SV_OK; ++d) {
        if (plans[d].empty()) continue;
        sv_state lead = owners[d][0];
        DeviceScope ds(lead->device);
        // The batch runs on the first state's stream, after the earlier work
        // queued on every state's own stream.
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            result = fail(SV_EDEVICE, "event creation failed");
            break;
        }
        for (sv_state o : owners[d]) {
            if (o->stream == lead->stream) continue;
            (void)hipEventRecord(ev, o->stream);
            (void)hipStreamWaitEvent(lead->stream, ev, 0);
        }
        sv_batch b = nullptr;
        result = sv_batch_create(d == 0 ? SV_C64 : SV_C128, lead->stream, &b);
        if (result == SV_OK) result = sv_batch_solo(b, 4096);   // 24+ qubits pass by pass
        if (result == SV_OK)
            result = sv_batch_run(b, plans[d].data(), nullptr, nullptr, plans[d].size(), flags & SV_GRAPH);
        if (b) {
            const sv_status sync = sv_batch_destroy(b);   // waits for the batch stream
            if (result == SV_OK) result = sync;
        }
        (void)hipEventDestroy(ev);
    }
    for (size_t k = 0; k < alone.size() && result == SV_OK; ++k) {
        const size_t c = alone[k];
        result = sv_run_circuit(states[c], circuits[c], lens[c], SV_FUSE);
        if (result == SV_OK) result = sv_synchronize(states[c]);
    }
    destroy_plans();
    return result;
}

sv_status sv_probs_device(sv_state s, uint64_t first, uint64_t count, double *out_dev)
{
    if (sv_status st = check_handle(s)) return st;
    const uint64_t N = uint64_t(1) << s->n;
    if (first > N || count > N - first)
        return fail(SV_EINVAL, "range [%llu, +%llu) exceeds 2^%d", (unsigned long long)first,
                    (unsigned long long)count, s->n);
    if (count == 0) return SV_OK;
    if (!out_dev) return fail(SV_EINVAL, "null output pointer");
    if (reinterpret_cast<uintptr_t>(out_dev) % 8 != 0)
        return fail(SV_EINVAL, "output pointer is not 8-byte aligned");
    DeviceScope ds(s->device);
    const int tok = svk::prof_begin(s);
    hipError_t e = svk::launch_probs(s->psi, s->dt, first, count, out_dev, s->stream);
    svk::prof_end(s, tok, svk::KC_PROBS, double(count) * (svk::elem_bytes(s->dt) + 8),
                  3.0 * double(count));
    if (e != hipSuccess) return hip_fail(e, "probs kernel launch");
    return SV_OK;
}

sv_status sv_probs(sv_state s, uint64_t first, uint64_t count, double *out_host)
{
    if (sv_status st = check_handle(s)) return st;
    const uint64_t N = uint64_t(1) << s->n;
    if (first > N || count > N - first)
        return fail(SV_EINVAL, "range [%llu, +%llu) exceeds 2^%d", (unsigned long long)first,
                    (unsigned long long)count, s->n);
    if (count == 0) return SV_OK;
    if (!out_host) return fail(SV_EINVAL, "null output pointer");
    DeviceScope ds(s->device);
    // Staged through a bounded device buffer so that a range of the largest
    // states never needs a second state-sized allocation.
    const uint64_t stage = std::min<uint64_t>(count, uint64_t(1) << 23);
    double *buf = nullptr;
    hipError_t e = hipMalloc(&buf, stage * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "hipMalloc of probs staging failed: %s", hipGetErrorString(e));
    }
    sv_status st = SV_OK;
    for (uint64_t off = 0; off < count && st == SV_OK; off += stage) {
        const uint64_t c = std::min(stage, count - off);
        e = svk::launch_probs(s->psi, s->dt, first + off, c, buf, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out_host + off, buf, c * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) st = hip_fail(e, "probs");
    }
    (void)hipFree(buf);
    return st;
}

sv_status sv_norm_device(sv_state s, double *out_dev)
{
    if (sv_status st = check_handle(s)) return st;
    if (!out_dev) return fail(SV_EINVAL, "null output pointer");
    DeviceScope ds(s->device);
    const int tok = svk::prof_begin(s);
    hipError_t e = svk::launch_norm(s->psi, s->n, s->dt, s->scratch, out_dev, s->stream);
    svk::prof_end(s, tok, svk::KC_NORM, double(state_bytes(s)), 4.0 * std::ldexp(1.0, s->n));
    if (e != hipSuccess) return hip_fail(e, "norm kernel launch");
    return SV_OK;
}

sv_status sv_norm(sv_state s, double *out)
{
    if (sv_status st = check_handle(s)) return st;
    if (!out) return fail(SV_EINVAL, "null output pointer");
    DeviceScope ds(s->device);
    double *res = s->scratch + svk::kNormBlocks;
    SV_HIP(svk::launch_norm(s->psi, s->n, s->dt, s->scratch, res, s->stream), "norm kernel launch");
    SV_HIP(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s->stream), "norm copy");
    SV_HIP(hipStreamSynchronize(s->stream), "norm synchronize");
    return SV_OK;
}

sv_status sv_compare(sv_state a, sv_state b, double out[4])
{
    if (sv_status st = check_handle(a)) return st;
    if (sv_status st = check_handle(b)) return st;
    if (!out) return fail(SV_EINVAL, "null output pointer");
    if (a->n != b->n) return fail(SV_EINVAL, "qubit counts differ (%d and %d)", a->n, b->n);
    if (a->device != b->device)
        return fail(SV_EINVAL, "states live on different devices (%d and %d)", a->device, b->device);
    DeviceScope ds(a->device);
    double *buf = nullptr;
    hipError_t e = hipMalloc(&buf, svk::kCompareScratch * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "hipMalloc of comparison scratch failed: %s", hipGetErrorString(e));
    }
    // The comparison runs on a's stream after the work queued so far on b's.
    hipEvent_t ev = nullptr;
    if (a->stream != b->stream) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, b->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(a->stream, ev, 0);
    }
    if (e == hipSuccess)
        e = svk::launch_compare(a->psi, a->dt, b->psi, b->dt, a->n, buf, a->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, buf + 4 * svk::kNormBlocks, 4 * sizeof(double),
                           hipMemcpyDeviceToHost, a->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
    if (ev) (void)hipEventDestroy(ev);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "state comparison");
    return SV_OK;
}

sv_status sv_copy_out(sv_state s, void *host_dst)
{
    if (sv_status st = check_handle(s)) return st;
    if (!host_dst) return fail(SV_EINVAL, "null host pointer");
    DeviceScope ds(s->device);
    SV_HIP(hipMemcpyAsync(host_dst, s->psi, state_bytes(s), hipMemcpyDeviceToHost, s->stream),
           "state copy out");
    SV_HIP(hipStreamSynchronize(s->stream), "copy-out synchronize");
    return SV_OK;
}

sv_status sv_copy_in(sv_state s, const void *host_src)
{
    if (sv_status st = check_handle(s)) return st;
    if (!host_src) return fail(SV_EINVAL, "null host pointer");
    DeviceScope ds(s->device);
    SV_HIP(hipMemcpyAsync(s->psi, host_src, state_bytes(s), hipMemcpyHostToDevice, s->stream),
           "state copy in");
    SV_HIP(hipStreamSynchronize(s->stream), "copy-in synchronize");
    return SV_OK;
}

sv_status sv_plan_inspect(int n_qubits, sv_dtype dtype, const sv_gate *gates, size_t n_gates,
                          uint32_t flags, int32_t *gate_op, int32_t *n_passes, int32_t *n_groups,
                          int32_t *n_ops)
{
    if (!valid_dtype(dtype)) return fail(SV_EINVAL, "unknown dtype %d", int(dtype));
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d not in [1, 34]", n_qubits);
    if (n_gates && !gates) return fail(SV_EINVAL, "null gate array");
    if ((flags & ~SV_NO_RELABEL) != SV_FUSE)
        return fail(SV_EUNSUPPORTED, "only SV_FUSE plans can be inspected");
    sv_state_s probe;
    probe.n = n_qubits;
    probe.dt = dtype;
    for (size_t i = 0; i < n_gates; ++i)
        if (sv_status st = validate_gate(&probe, gates[i], i)) return st;
    if (svk::plan_inspect(n_qubits, dtype, gates, n_gates, !(flags & SV_NO_RELABEL), gate_op, n_passes,
                          n_groups, n_ops) != 0)
        return fail(SV_EUNSUPPORTED, "planner could not place every gate with this tile geometry");
    return SV_OK;
}

sv_status sv_plan_jit_check(int n_qubits, sv_dtype dtype, const sv_gate *gates, size_t n_gates,
                            uint32_t flags, int32_t *n_programs)
{
    if (!valid_dtype(dtype)) return fail(SV_EINVAL, "unknown dtype %d", int(dtype));
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d not in [1, 34]", n_qubits);
    if (n_gates && !gates) return fail(SV_EINVAL, "null gate array");
    if ((flags & ~SV_NO_RELABEL) != (SV_FUSE | SV_JIT))
        return fail(SV_EINVAL, "flags must be SV_FUSE | SV_JIT, optionally | SV_NO_RELABEL");
    sv_state_s probe;
    probe.n = n_qubits;
    probe.dt = dtype;
    for (size_t i = 0; i < n_gates; ++i)
        if (sv_status st = validate_gate(&probe, gates[i], i)) return st;
    std::string err;
    const int rc = svk::plan_jit_check(n_qubits, dtype, gates, n_gates, !(flags & SV_NO_RELABEL),
                                       n_programs, &err);
    if (rc == -1) return fail(SV_EUNSUPPORTED, "%s", err.c_str());
    if (rc != 0) return fail(SV_EDEVICE, "%s", err.c_str());
    return SV_OK;
}

sv_status sv_plan_dense_inspect(int n_qubits, const sv_gate *gates, size_t n_gates,
                                uint64_t *block_masks, double *block_mats, int32_t cap,
                                int32_t *n_blocks)
{
    if (n_qubits < 5 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d not in [5, 34]", n_qubits);
    if (n_gates && !gates) return fail(SV_EINVAL, "null gate array");
    if (cap < 0) return fail(SV_EINVAL, "negative capacity");
    sv_state_s probe;
    probe.n = n_qubits;
    for (size_t i = 0; i < n_gates; ++i)
        if (sv_status st = validate_gate(&probe, gates[i], i)) return st;
    if (sv_status st = reject_wide(gates, n_gates)) return st;
    const int nb = svk::plan_dense_inspect(n_qubits, gates, n_gates, block_masks, block_mats, cap);
    if (n_blocks) *n_blocks = nb;
    return SV_OK;
}

sv_status sv_plan_create(sv_state s, const sv_gate *gates, size_t n_gates, sv_plan *out)
{
    if (sv_status st = check_handle(s)) return st;
    if (!out) return fail(SV_EINVAL, "null output pointer");
    *out = nullptr;
    if (n_gates && !gates) return fail(SV_EINVAL, "null gate array");
    for (size_t i = 0; i < n_gates; ++i)
        if (sv_status st = validate_gate(s, gates[i], i)) return st;
    DeviceScope ds(s->device);
    std::string err;
    sv_status st = svk::plan_create(s, gates, n_gates, out, &err);
    if (st != SV_OK) return fail(st, "%s", err.c_str());
    return SV_OK;
}

sv_status sv_synchronize(sv_state s)
{
    if (sv_status st = check_handle(s)) return st;
    DeviceScope ds(s->device);
    SV_HIP(hipStreamSynchronize(s->stream), "stream synchronize");
    return SV_OK;
}

sv_status sv_sample_device(sv_state s, const double *u_dev, uint64_t count, uint64_t *out_dev)
{
    if (sv_status st = check_handle(s)) return st;
    if (count == 0) return SV_OK;
    if (!u_dev || !out_dev) return fail(SV_EINVAL, "null device pointer");
    DeviceScope ds(s->device);
    const uint64_t need = svk::sample_scratch_doubles(s->n);
    if (s->sample_cap < need) {
        if (s->sample_scratch) {
            SV_HIP(hipStreamSynchronize(s->stream), "stream synchronize");
            (void)hipFree(s->sample_scratch);
            s->sample_scratch = nullptr;
            s->sample_cap = 0;
        }
        hipError_t e = hipMalloc(&s->sample_scratch, need * sizeof(double));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SV_ENOMEM, "hipMalloc of sampling scratch failed: %s", hipGetErrorString(e));
        }
        s->sample_cap = need;
    }
    const double N = std::ldexp(1.0, s->n), sb = svk::elem_bytes(s->dt);
    const int tok = svk::prof_begin(s);
    hipError_t e = svk::launch_block_sums(s->psi, s->n, s->dt, s->sample_scratch, s->stream);
    if (e == hipSuccess)
        e = svk::launch_sample(s->psi, s->n, s->dt, s->sample_scratch, u_dev, count, out_dev,
                               s->stream);
    // algorithmic bytes: the state once, the draws and the indices
    svk::prof_end(s, tok, svk::KC_SAMPLE, N * sb + double(count) * 16.0, 3.0 * N);
    if (e != hipSuccess) return hip_fail(e, "sampling kernel launch");
    return SV_OK;
}

sv_status sv_sample_device_noalloc(sv_state s, const double *u_dev, uint64_t count,
                                   uint64_t *out_dev)
{
    if (sv_status st = check_handle(s)) return st;
    if (s->n > svk::kStaticSampleMaxQubits)
        return fail(SV_EINVAL, "n = %d exceeds the %d qubits the static sampling scratch serves "
                    "(sv_sample_device takes any n)", s->n, svk::kStaticSampleMaxQubits);
    if (count == 0) return SV_OK;
    if (!u_dev || !out_dev) return fail(SV_EINVAL, "null device pointer");
    DeviceScope ds(s->device);
    double *S = nullptr;
    SV_HIP(svk::static_sample_scratch(s->device, &S), "static sampling scratch lookup");
    // Every scratch entry the launches read is written by them first (block
    // sums, then their prefix), so nothing is cleared between calls.
    SV_HIP(svk::launch_block_sums(s->psi, s->n, s->dt, S, s->stream), "block-sum kernel launch");
    SV_HIP(svk::launch_sample(s->psi, s->n, s->dt, S, u_dev, count, out_dev, s->stream),
           "sampling kernel launch");
    return SV_OK;
}

}  // extern "C"
