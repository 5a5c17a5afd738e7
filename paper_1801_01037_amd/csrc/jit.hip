// Tile passes compiled for their own program (SV_JIT).
//
// The generic tile kernel reads each op of a pass from its device record and
// dispatches on the op's kind and register positions at run time: scalar
// loads and branches before every op, and, since its ops alternate between
// two register arrays inside a loop, a register copy for every amplitude an
// op leaves unchanged. Here a pass's program -- its groups' register bits and
// its ops' kinds, register positions and controls -- is written out as the
// body of a kernel of its own and compiled with hipRTC: every op is a call
// of the same device function the generic kernel uses (tile_dev.h), with its
// positions as template arguments, in straight-line code, so the compiler
// renames registers instead of copying them, resolves every control position
// and loads the op matrices ahead of their use. The numbers the ops read
// (matrices, diagonal tables) stay in the plan's device records, so one
// compiled program serves every pass of the same shape; kernels are cached per
// device and program text for the life of the process.
//
// What is known when a program is written out is also used to do less work:
// a diagonal op skips the phases that its shape makes exactly 1 (a controlled
// phase on a register bit touches half of the amplitudes), a real 2x2 (a
// Hadamard) skips its zero imaginary parts, and the first and last groups
// move the tile between HBM and registers directly, without an LDS round
// trip, when their register bits leave the tile's low index bits to the
// threads. None of this changes a result bit.
//
// A compiled program that would spill registers to scratch memory is not
// used: its pass runs with the generic kernel.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>
#include <utility>
#include <vector>

#include "plan.h"
#include "sv_internal.h"
#include "tile.h"

// kTileHSrc, kTileDevHSrc: the text of tile.h and tile_dev.h, written by the
// build next to the objects.
#include "jit_src.inc"

namespace svk {
namespace {

int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}
const int kJitWavesC128 = env_int("SV_JIT_WAVES128", 2);
const int kJitWavesC64 = env_int("SV_JIT_WAVES64", 4);

// Output local bit that input local bit s is written to: the pass's
// relabelled order when it has one.
int out_bit(const TileArgs &a, int s)
{
    if (a.permute)
        for (int j = 0; j < a.L; ++j)
            if (int((a.osrc >> (4 * j)) & 15u) == s) return j;
    return s;
}

// The first group loads its registers straight from HBM when the threads'
// own bits hold the tile's low nlow bits (then 2^nlow neighbouring threads
// read one aligned run of amplitudes); the last group stores straight to HBM
// when the same holds for the bits it writes to.
bool direct_first(const TileArgs &a, const TileGroup &G, int K)
{
    for (int k = 0; k < K; ++k)
        if (G.s[k] < a.nlow) return false;
    return true;
}

bool direct_last(const TileArgs &a, const TileGroup &G, int K)
{
    for (int k = 0; k < a.nlow && k < a.L - K; ++k)
        if (out_bit(a, G.ns[k]) >= a.nlow) return false;
    return true;
}

const bool kJitDirect = env_int("SV_JIT_DIRECT", 1) != 0;


// Register combination that combination r of group G is written back as: its
// exit map (TileGroup), or r itself.
uint32_t exit_of(const TileGroup &G, int K, int r)
{
    if (!G.has_exit) return uint32_t(r);
    uint32_t x = G.xb;
    for (int k = 0; k < K; ++k)
        if (r & (1 << k)) x ^= G.xs[k];
    return x;
}


std::string pass_source(const TileArgs &a, const TileGroup *groups, const TileOp *ops, int K,
                        bool c64, bool nt)
{
    const int L = a.L;
    const uint32_t size = 1u << L;
    const uint32_t slots = tile_slots(c64, size);
    const int threads = 1 << (L - K);
    const int NR = 1 << K;
    const int ng = a.ngroups;
    const bool df = kJitDirect && ng > 0 && direct_first(a, groups[0], K);
    const bool dl = kJitDirect && ng > 0 && direct_last(a, groups[ng - 1], K);
    std::ostringstream o;
    // Resident waves per SIMD the code is built for: the LDS of a work-group
    // allows two complex128 tiles per CU (two waves per SIMD); complex64
    // tiles leave room for more. Straight-line programs otherwise let the
    // scheduler hoist loads far ahead and hold hundreds of registers.
    const int waves = c64 ? kJitWavesC64 : kJitWavesC128;
    o << "#include \"tile_dev.h\"\n"
         "using namespace svk;\nusing namespace svk::dev;\n"
         "extern \"C\" __global__ __launch_bounds__("
      << threads << ") __attribute__((amdgpu_waves_per_eu(" << waves
      << "))) void svj_pass(TileArgs a)\n{\n";
    o << "    constexpr bool C64 = " << (c64 ? "true" : "false") << ";\n"
      << "    constexpr int K = " << K << ";\n"
      << "    using A = AmpT<C64>;\n"
      << "    __shared__ __align__(16) A smem[" << slots << " + 512];\n"
      << "    A *lds = smem;\n"
      << "    A *tab = smem + " << slots << ";\n"
      << "    CGroup *groups = (CGroup *)(a.groups) + a.group0;\n";
    // A pass that only restores the storage order has no group (and no op).
    const int op_base = ng > 0 ? groups[0].op0 : 0;
    if (ng > 0) o << "    COp *ops = (COp *)(a.ops) + groups[0].op0;\n";
    // Direct transfers: each thread's own index bits (the same for every
    // tile) and the index bits of the register bits, computed once.
    if (df || dl) o << "    const uint32_t t0 = threadIdx.x;\n";
    if (df) {
        const TileGroup &G = groups[0];
        o << "    const uint64_t dfirst = deposit(0u";
        for (int k = 0; k < L - K; ++k) o << " | (((t0 >> " << k << ") & 1u) << " << G.ns[k] << ")";
        o << ", a.tmask);\n    const uint64_t rbf[K] = {";
        for (int k = 0; k < K; ++k) o << (k ? ", " : "") << "nth_bit(a.tmask, " << G.s[k] << ")";
        o << "};\n";
    }
    if (dl) {
        const TileGroup &G = groups[ng - 1];
        o << "    const uint64_t dlast = deposit(0u";
        for (int k = 0; k < L - K; ++k)
            o << " | (((t0 >> " << k << ") & 1u) << " << out_bit(a, G.ns[k]) << ")";
        o << ", a.tmask);\n    const uint64_t obl[K] = {";
        for (int k = 0; k < K; ++k) o << (k ? ", " : "") << "nth_bit(a.tmask, " << out_bit(a, G.s[k]) << ")";
        o << "};\n    const uint32_t xrl[1 << K] = {";
        for (int r = 0; r < NR; ++r) o << (r ? ", " : "") << exit_of(G, K, r) << "u";
        o << "};\n";
    }
    // tid is made opaque at every group, so that nothing derived from it (slot
    // addresses, per-thread diagonal rows) is hoisted out of the tile loop
    // and held in registers through all the tiles. Every thread of the
    // work-group holds amplitudes (2^(L-K) threads).
    o << "    auto prog = [&](uint64_t g, uint64_t gbase, const Walk<K> &w, const A (&cur)[1 << K]) {\n";
    for (int gi = 0; gi < ng; ++gi) {
        const TileGroup &G = groups[gi];
        const bool first = gi == 0 && df, last = gi == ng - 1 && dl;
        o << "        {\n"
          << "            CGroup &G = groups[" << gi << "];\n"
          << "            uint32_t tid = w.tid;\n"
          << "            asm volatile(\"\" : \"+v\"(tid));\n"
          << "            __builtin_amdgcn_s_setprio(2);\n"
          << "            const uint32_t lbase = 0u";
        for (int k = 0; k < L - K; ++k) o << " | (((tid >> " << k << ") & 1u) << " << G.ns[k] << ")";
        o << ";\n            const uint32_t soff[K] = {";
        for (int k = 0; k < K; ++k) o << (k ? ", " : "") << (1u << G.s[k]) << "u";
        o << "};\n"
          << "            A v[1 << K], u[1 << K];\n";
        if (first)
            o << "            take_regs<C64, K>(cur, v);\n";
        else
            o << "            gather_fixed<C64, K>(lds, lbase, soff, v);\n";
        const char *arr[2] = {"v", "u"};
        for (int oi = 0; oi < G.nops; ++oi) {
            const TileOp &t = ops[G.op0 + oi];
            const int k = G.op0 + oi - op_base;
            const char *in = arr[oi & 1], *out = arr[(oi + 1) & 1];
            std::ostringstream core;
            if (t.kind == TOP_DIAG) {
                // A diagonal op's phases depend only on the thread and the
                // tile, so the compiler would evaluate those of every
                // diagonal op of a group up front and hold them all (about 64
                // registers each). Tying the thread index to all of the op's
                // input amplitudes makes it evaluate them when the op runs.
                core << "{ uint32_t dtid = tid; asm volatile(\"\" : \"+v\"(dtid) :";
                for (int r = 0; r < NR; ++r) core << (r ? ", " : " ") << "\"v\"(" << in << "[" << r << "].x)";
                // The op's shape: phases that are exactly 1 are skipped.
                uint32_t one = 0;
                for (int r = 0; r < NR; ++r)
                    if (!t.pj || (t.m4[2 * r] == 1.0 && t.m4[2 * r + 1] == 0.0)) one |= 1u << r;
                core << "); apply_diag_shape<C64, K, " << (t.dlin & ((1u << K) - 1)) << "u, "
                     << ((t.dlin & kDiagBase) ? "true" : "false") << ", " << one << "u>(" << in
                     << ", " << out << ", ops[" << k << "], a.dtab, a.L, G, g, dtid, tab); }";
            } else if (t.kind == TOP_U4) {
                core << "u4_pp<C64, K, " << t.pj << ", " << t.pk << ">(" << in << ", " << out
                     << ", ops[" << k << "]);";
            } else {
                const char *sw = t.kind == TOP_SWAP ? "true" : "false";
                if (t.pk >= 0)
                    core << "pair_rc<C64, K, " << t.pj << ", " << t.pk << ", " << sw << ">(" << in
                         << ", " << out << ", ops[" << k << "]);";
                else {
                    const bool real = t.kind == TOP_U && t.m[1] == 0.0 && t.m[3] == 0.0 &&
                                      t.m[5] == 0.0 && t.m[7] == 0.0;
                    core << "pair_pj<C64, K, " << t.pj << ", " << sw << ", "
                         << ((t.lctrl >= 0 || t.lcm) ? "true" : "false") << ", "
                         << (real ? "true" : "false") << ">(" << in << ", " << out << ", lbase, soff, ops["
                         << k << "]);";
                }
            }
            std::string cond;
            if (t.kind != TOP_DIAG && t.kind != TOP_U4) {
                if (t.octrl >= 0) cond = "((gbase >> " + std::to_string(t.octrl) + ") & 1ull)";
                if (t.ocm) {
                    const std::string m = std::to_string(t.ocm) + "ull";
                    cond = (cond.empty() ? "" : cond + " && ") + "((gbase & " + m + ") == " + m + ")";
                }
            }
            // Ops are scheduled one after the other: hoisting an op's matrix
            // loads over the op before it holds two matrices in scalar
            // registers (64 each for a 4x4) and spills them to vector lanes.
            if (oi > 0) o << "            __builtin_amdgcn_sched_barrier(0);\n";
            if (cond.empty())
                o << "            " << core.str() << "\n";
            else
                o << "            if (" << cond << ") " << core.str() << "\n"
                  << "            else copy_amps<C64, K>(" << in << ", " << out << ");\n";
        }
        const char *fin = arr[G.nops & 1];
        if (last) {
            if (first) {
                // One group, loaded and stored directly: every load of the
                // tile has returned before a store may overwrite its
                // amplitude (a relabelled store writes other threads' ones,
                // so the whole work-group waits).
                o << "            asm volatile(\"\" : :";
                for (int r = 0; r < NR; ++r) o << (r ? ", " : " ") << "\"v\"(v[" << r << "].x)";
                o << ");\n";
                if (a.permute) o << "            lds_barrier();\n";
            }
            o << "            store_direct<C64, K, " << (nt ? "true" : "false")
              << ">(a, gbase | dlast, obl, xrl, " << fin << ");\n"
              << "            __builtin_amdgcn_s_setprio(0);\n"
              << "        }\n";
            continue;
        }
        // A first group that loaded from HBM writes slots that other threads
        // of the previous tile may still be reading.
        if (first) o << "            lds_barrier();\n";
        if (G.has_exit) {
            // the exit map as constants: every slot offset is an immediate
            o << "            const uint32_t xr[1 << K] = {";
            for (int r = 0; r < NR; ++r) o << (r ? ", " : "") << exit_of(G, K, r) << "u";
            o << "};\n            write_map<C64, K>(lds, " << fin << ", lbase, soff, xr);\n";
        } else {
            o << "            scatter_fixed<C64, K>(lds, " << fin << ", lbase, soff);\n";
        }
        o << "            __builtin_amdgcn_s_setprio(0);\n"
          << "            lds_barrier();\n"
          << "        }\n";
    }
    o << "    };\n";
    // A direct first group's fetch: in its own layout.
    if (df)
        o << "    auto fetch = [&](uint64_t gb, const Walk<K> &, A (&p)[1 << K]) {\n"
          << "        fetch_direct<C64, K, " << (nt ? "true" : "false") << ">(a, gb | dfirst, rbf, p);\n"
          << "    };\n";
    else
        o << "    NoFetch fetch;\n";
    // Each work-group walks a contiguous range of tiles: the stores of one
    // tile and the loads of the next fall on neighbouring lines.
    o << "    const uint64_t per = (a.ntiles + gridDim.x - 1) / gridDim.x;\n"
      << "    const uint64_t t0b = uint64_t(blockIdx.x) * per;\n"
      << "    const uint64_t t1b = t0b + per < a.ntiles ? t0b + per : a.ntiles;\n"
      << "    walk_tiles<C64, K, " << (nt ? "true" : "false") << ", " << (df ? "true" : "false")
      << ", " << (dl ? "true" : "false") << ">(a, t0b, t1b, 1, lds, tab, prog, fetch);\n}\n";
    if (std::getenv("SV_JIT_VERBOSE"))
        std::fprintf(stderr, "[sv jit] pass: %d groups, direct first %d, direct last %d, permute %d\n",
                     ng, int(df), int(dl), int(a.permute));
    return o.str();
}

struct Compiled {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int per_cu = 1;     // resident work-groups per CU
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, Compiled> g_cache;

// Compiles one program; the code object in *code, or the log in *err.
bool compile(const std::string &src, std::vector<char> *code, std::string *err)
{
    hiprtcProgram prog = nullptr;
    const char *hdrs[2] = {kTileHSrc, kTileDevHSrc};
    const char *names[2] = {"tile.h", "tile_dev.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "svj_pass.hip", 2, hdrs, names) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return false;
    }
    // The library's own build flags: no packed FP32 instructions, and no
    // sinking of switch arms into selects over register arrays.
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-mllvm", "-simplifycfg-sink-common=false"};
    const hiprtcResult r = hiprtcCompileProgram(prog, int(sizeof opts / sizeof opts[0]), opts);
    bool ok = r == HIPRTC_SUCCESS;
    if (ok) {
        size_t n = 0;
        ok = hiprtcGetCodeSize(prog, &n) == HIPRTC_SUCCESS && n > 0;
        if (ok) {
            code->resize(n);
            ok = hiprtcGetCode(prog, code->data()) == HIPRTC_SUCCESS;
        }
    }
    if (!ok) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
        }
        *err = std::string("run-time compilation of a tile pass failed: ") +
               hiprtcGetErrorString(r) + "\n" + log;
    }
    (void)hiprtcDestroyProgram(&prog);
    // SV_JIT_DUMP=<directory>: keep each program's text and code object there
    // (for reading the generated code; the library never reads them back).
    if (const char *dir = std::getenv("SV_JIT_DUMP")) {
        const std::string stem = std::string(dir) + "/svj_" + std::to_string(std::hash<std::string>{}(src));
        if (FILE *f = std::fopen((stem + ".hip").c_str(), "w")) {
            std::fwrite(src.data(), 1, src.size(), f);
            std::fclose(f);
        }
        if (ok)
            if (FILE *f = std::fopen((stem + ".co").c_str(), "wb")) {
                std::fwrite(code->data(), 1, code->size(), f);
                std::fclose(f);
            }
    }
    return ok;
}

int cus_of_device()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

}  // namespace

sv_status jit_passes(sv_dtype dt, int K, const std::vector<TileArgs> &passes,
                     const std::vector<TileGroup> &groups, const std::vector<TileOp> &ops,
                     std::vector<JitKernel> *out, std::string *err)
{
    const bool c64 = dt == SV_C64;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::vector<std::string> srcs(passes.size());
    for (size_t p = 0; p < passes.size(); ++p) {
        const TileArgs &a = passes[p];
        const bool nt = (a.ntiles << a.L) * uint64_t(c64 ? 8 : 16) > kStreamBytes;
        srcs[p] = pass_source(a, a.ngroups > 0 ? groups.data() + a.group0 : nullptr, ops.data(), K,
                              c64, nt);
    }
    // Programs not compiled yet on this device, each once.
    std::vector<std::string> todo;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (const std::string &s : srcs)
            if (!s.empty() && !g_cache.count({dev, s}) &&
                std::find(todo.begin(), todo.end(), s) == todo.end())
                todo.push_back(s);
    }
    std::vector<std::vector<char>> codes(todo.size());
    std::vector<std::string> errs(todo.size());
    std::vector<char> ok(todo.size(), 0);
    {
        const size_t nthr = std::max<size_t>(
            1, std::min<size_t>({todo.size(), size_t(std::max(1u, std::thread::hardware_concurrency())),
                                 size_t(16)}));
        std::vector<std::thread> pool;
        for (size_t t = 0; t < nthr; ++t)
            pool.emplace_back([&, t]() {
                for (size_t i = t; i < todo.size(); i += nthr)
                    ok[i] = compile(todo[i], &codes[i], &errs[i]) ? 1 : 0;
            });
        for (std::thread &th : pool) th.join();
    }
    for (size_t i = 0; i < todo.size(); ++i) {
        if (!ok[i]) {
            *err = errs[i];
            return SV_EDEVICE;
        }
        Compiled c;
        hipError_t e = hipModuleLoadData(&c.mod, codes[i].data());
        if (e == hipSuccess) e = hipModuleGetFunction(&c.fn, c.mod, "svj_pass");
        int scratch = 0;
        if (e == hipSuccess &&
            hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, c.fn) != hipSuccess)
            scratch = 0;
        if (std::getenv("SV_JIT_VERBOSE"))
            std::fprintf(stderr, "[sv jit] program %zu: %zu bytes of code, load %s, scratch %d bytes\n",
                         std::hash<std::string>{}(todo[i]), codes[i].size(), hipGetErrorString(e),
                         scratch);
        if (e == hipSuccess && scratch > 0) {
            // spills registers: the generic kernel runs such passes
            (void)hipModuleUnload(c.mod);
            c = Compiled{};
        } else if (e == hipSuccess) {
            // every pass of a dtype has the same tile bits, hence threads
            const int threads = 1 << (passes[0].L - K);
            int n = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, c.fn, threads, 0) != hipSuccess ||
                n <= 0) {
                (void)hipGetLastError();
                n = 1;
            }
            c.per_cu = n;
        }
        if (e != hipSuccess) {
            if (c.mod) (void)hipModuleUnload(c.mod);
            *err = std::string("loading a compiled tile pass: ") + hipGetErrorString(e);
            return SV_EDEVICE;
        }
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_cache.emplace(std::make_pair(dev, todo[i]), c).second) (void)hipModuleUnload(c.mod);
    }
    out->clear();
    std::lock_guard<std::mutex> lock(g_mu);
    for (size_t p = 0; p < passes.size(); ++p) {
        if (srcs[p].empty()) {
            out->push_back(JitKernel{nullptr, 0});
            continue;
        }
        const Compiled &c = g_cache.at({dev, srcs[p]});
        out->push_back(JitKernel{c.fn, c.per_cu});
    }
    return SV_OK;
}

bool jit_compile_only(sv_dtype dt, int K, const std::vector<TileArgs> &passes,
                      const std::vector<TileGroup> &groups, const std::vector<TileOp> &ops,
                      int32_t *n_programs, std::string *err)
{
    const bool c64 = dt == SV_C64;
    std::vector<std::string> srcs;
    for (const TileArgs &a : passes) {
        const bool nt = (a.ntiles << a.L) * uint64_t(c64 ? 8 : 16) > kStreamBytes;
        std::string s = pass_source(a, a.ngroups > 0 ? groups.data() + a.group0 : nullptr,
                                    ops.data(), K, c64, nt);
        if (std::find(srcs.begin(), srcs.end(), s) == srcs.end()) srcs.push_back(std::move(s));
    }
    std::vector<char> code;
    for (const std::string &s : srcs)
        if (!compile(s, &code, err)) return false;
    if (n_programs) *n_programs = int32_t(srcs.size());
    return true;
}

hipError_t jit_launch(const JitKernel &k, const TileArgs &a, int K, bool c64, hipStream_t st)
{
    if (!k.fn) return launch_tile(a, K, c64, st);   // a pass left to the generic kernel
    static const int cus = cus_of_device();
    const unsigned threads = 1u << (a.L - K);
    const uint64_t want = uint64_t(cus) * uint64_t(k.per_cu);
    const unsigned grid = unsigned(a.ntiles < want ? a.ntiles : want);
    TileArgs arg = a;
    void *params[] = {&arg};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, threads, 1, 1, 0, st, params, nullptr);
}

}  // namespace svk
