// SV_GRAPH for sv_run_circuit: the launches of one circuit on one state,
// captured once in a HIP graph and replayed.
//
// A circuit run again and again (a serving loop, a benchmark step) pays the
// host cost of planning and of every launch each time. With SV_GRAPH the
// first run plans the gate list, uploads what its kernels read (tile plans,
// dense block matrices) into buffers that belong to the graph, and captures the
// launches alone on a private stream -- no copies and no memsets are recorded,
// so a replay is kernels only. Later runs of the same gate list with the same
// flags replay the graph on the handle's stream. One graph is kept per handle;
// a different gate list or different flags replace it.
//
// The captured launches are the ones the same flags queue without SV_GRAPH:
// tile passes (relabelled unless SV_NO_RELABEL) for SV_FUSE, dense 5-qubit
// blocks for SV_FUSE_DENSE (n >= 9; tile passes below), one launch per gate
// for SV_GRAPH alone, and one launch per gate of more than five qubits between
// dense segments. Results are bit for bit those of the same flags without
// SV_GRAPH.
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.h"
#include "sv_internal.h"

namespace svk {
namespace {

// One step of a captured run: a planned tile segment, a dense segment, or a
// single gate.
struct Step {
    enum Kind { TILES, DENSE, GATE } kind;
    size_t first = 0, last = 0;         // TILES, DENSE: launches [first, last)
    int K = 4;                          // TILES: register bits of the passes
    sv_gate gate{};                     // GATE
};

struct CircuitGraph {
    std::vector<sv_gate> gates;         // the list the graph was captured for
    uint32_t flags = 0;
    void *psi = nullptr;
    std::vector<Step> steps;
    std::vector<void *> bufs;           // tile tables and block matrices the graph reads
    std::vector<TileArgs> tiles;
    std::vector<JitKernel> jit;         // SV_JIT: the compiled kernel of each of `tiles`
    std::vector<DenseArgs> dense;
    hipStream_t capture = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;         // stream of the last replay
    double bytes = 0.0, flops = 0.0;    // algorithmic, per replay (profiling)

    void free_buffers()
    {
        for (void *d : bufs) (void)hipFree(d);
        bufs.clear();
        tiles.clear();
        jit.clear();
        dense.clear();
        steps.clear();
    }
};

bool same_gates(const std::vector<sv_gate> &a, const sv_gate *b, size_t n)
{
    return a.size() == n && (n == 0 || std::memcmp(a.data(), b, n * sizeof(sv_gate)) == 0);
}

// Plans the segments of the gate list into steps; every device buffer the
// steps read is uploaded here, before any capture.
sv_status build_steps(sv_state s, CircuitGraph *g, const sv_gate *gates, size_t n_gates,
                      uint32_t flags, std::string *err)
{
    const double N = std::ldexp(1.0, s->n), sb = elem_bytes(s->dt);
    const bool fuse = flags & (SV_FUSE | SV_FUSE_DENSE);
    const bool dense = (flags & SV_FUSE_DENSE) && s->n >= 9;
    // As without SV_GRAPH: dense blocks hold at most five qubits, so a wider
    // gate with several controls is a launch of its own there.
    auto alone = [&](const sv_gate &g) {
        if (!fuse) return true;
        if (!dense || g.kind != SV_G_MCU) return false;
        const uint64_t cm = uint64_t(uint32_t(g.control)) | (uint64_t(uint32_t(g.flags)) << 32);
        return __builtin_popcountll(cm) + 1 > 5;
    };
    size_t i = 0;
    while (i < n_gates) {
        if (alone(gates[i])) {
            Step st;
            st.kind = Step::GATE;
            st.gate = gates[i];
            g->steps.push_back(st);
            g->bytes += 2.0 * N * sb;   // at most one full pass per gate
            ++i;
            continue;
        }
        size_t j = i;
        while (j < n_gates && !alone(gates[j])) ++j;
        Step st;
        void *dev = nullptr;
        if ((flags & SV_FUSE_DENSE) && s->n >= 9) {
            std::vector<DenseArgs> blocks;
            if (sv_status r = dense_prepare(s, gates + i, j - i, &dev, &blocks, err)) return r;
            st.kind = Step::DENSE;
            st.first = g->dense.size();
            g->dense.insert(g->dense.end(), blocks.begin(), blocks.end());
            st.last = g->dense.size();
            g->flops += 256.0 * N * double(blocks.size());
        } else {
            std::vector<TileArgs> passes;
            std::vector<JitKernel> kern;
            if (sv_status r = tiles_prepare(s, gates + i, j - i, !(flags & SV_NO_RELABEL), &dev,
                                            &passes, &st.K, (flags & SV_JIT) ? &kern : nullptr, err))
                return r;
            st.kind = Step::TILES;
            st.first = g->tiles.size();
            g->tiles.insert(g->tiles.end(), passes.begin(), passes.end());
            if (flags & SV_JIT) g->jit.insert(g->jit.end(), kern.begin(), kern.end());
            st.last = g->tiles.size();
        }
        g->bufs.push_back(dev);
        g->steps.push_back(st);
        g->bytes += 2.0 * N * sb * double(st.last - st.first);
        i = j;
    }
    return SV_OK;
}

// Queues every step on s->stream (the capture stream while capturing).
sv_status queue_steps(sv_state s, const CircuitGraph &g, std::string *err)
{
    const bool c64 = s->dt == SV_C64;
    for (const Step &st : g.steps) {
        hipError_t e = hipSuccess;
        switch (st.kind) {
        case Step::TILES:
            for (size_t p = st.first; p < st.last && e == hipSuccess; ++p)
                e = g.jit.empty() ? launch_tile(g.tiles[p], st.K, c64, s->stream)
                                  : jit_launch(g.jit[p], g.tiles[p], st.K, c64, s->stream);
            break;
        case Step::DENSE:
            for (size_t b = st.first; b < st.last && e == hipSuccess; ++b)
                e = launch_dense5(g.dense[b], c64, s->stream);
            break;
        case Step::GATE:
            if (sv_status r = queue_gate(s, st.gate)) {
                *err = sv_last_error();
                return r;
            }
            break;
        }
        if (e != hipSuccess) {
            *err = std::string("launch while capturing: ") + hipGetErrorString(e);
            return SV_EDEVICE;
        }
    }
    return SV_OK;
}

sv_status capture(sv_state s, CircuitGraph *g, std::string *err)
{
    if (!g->capture) {
        hipError_t e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            g->capture = nullptr;
            *err = std::string("capture stream: ") + hipGetErrorString(e);
            return SV_EDEVICE;
        }
    }
    hipError_t e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        *err = std::string("begin capture: ") + hipGetErrorString(e);
        return SV_EDEVICE;
    }
    // The steps queue on the handle's stream and time themselves when
    // profiling is on: point the handle at the capture stream and pause
    // profiling while they are recorded.
    const hipStream_t user = s->stream;
    const bool prof = s->prof.on;
    s->stream = g->capture;
    s->prof.on = false;
    sv_status st = queue_steps(s, *g, err);
    s->stream = user;
    s->prof.on = prof;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->capture, &graph);
    if (st != SV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) {
        *err = std::string("end capture: ") + hipGetErrorString(e);
        return SV_EDEVICE;
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g->exec = nullptr;
        *err = std::string("graph instantiate: ") + hipGetErrorString(e);
        return SV_EDEVICE;
    }
    return SV_OK;
}

void drop(CircuitGraph *g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);   // callers have waited for its replays
    g->exec = nullptr;
    g->free_buffers();
    g->gates.clear();
}

}  // namespace

sv_status circuit_graph_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                            std::string *err)
{
    if (!s->graph) s->graph = new CircuitGraph();
    CircuitGraph *g = static_cast<CircuitGraph *>(s->graph);
    const uint32_t key = flags & (SV_FUSE | SV_FUSE_DENSE | SV_NO_RELABEL | SV_JIT);
    if (!g->exec || g->flags != key || g->psi != s->psi || !same_gates(g->gates, gates, n_gates)) {
        if (g->exec) {
            // Replays of the old graph may still be queued; they read the
            // buffers about to be freed.
            hipError_t e = hipStreamSynchronize(g->last);
            if (e != hipSuccess) {
                *err = std::string("stream synchronize: ") + hipGetErrorString(e);
                return SV_EDEVICE;
            }
        }
        drop(g);
        g->bytes = g->flops = 0.0;
        sv_status st = build_steps(s, g, gates, n_gates, key, err);
        if (st == SV_OK) st = capture(s, g, err);
        if (st != SV_OK) {
            drop(g);
            return st;
        }
        g->gates.assign(gates, gates + n_gates);
        g->flags = key;
        g->psi = s->psi;
    }
    const int tok = prof_begin(s);
    hipError_t e = hipGraphLaunch(g->exec, s->stream);
    g->last = s->stream;
    prof_end(s, tok, KC_GRAPH, g->bytes, g->flops);
    if (e != hipSuccess) {
        *err = std::string("graph launch: ") + hipGetErrorString(e);
        return SV_EDEVICE;
    }
    return SV_OK;
}

void circuit_graph_release(sv_state s)
{
    if (!s->graph) return;
    CircuitGraph *g = static_cast<CircuitGraph *>(s->graph);
    if (g->exec) (void)hipStreamSynchronize(g->last);
    drop(g);
    if (g->capture) (void)hipStreamDestroy(g->capture);
    delete g;
    s->graph = nullptr;
}

}  // namespace svk
