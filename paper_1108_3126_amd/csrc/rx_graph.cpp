// Replay of a batched call's launch sequence from a captured HIP graph.
//
// A batched match is a fixed sequence of launches (sort or bucket, gather,
// circuits or items, results); with the same shape it differs from call to
// call only in its pointers and sizes.  The sequence is recorded once by
// stream capture on a private stream (nothing runs there), instantiated, and
// replayed on the caller's stream; a call whose arguments changed records the
// sequence again and updates the instantiated graph in place when the launch
// topology is unchanged, else instantiates anew.  A few graphs are kept per
// device (least recently used go first).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "rx_internal.h"

namespace rx {
namespace {

constexpr int kGraphsPerDevice = 8;

struct GraphEntry {
    std::string topo, full;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;   // recorded after the latest replay
    uint64_t used = 0;
};

struct DeviceGraphs {
    hipStream_t capture = nullptr;
    std::vector<GraphEntry> entries;
    uint64_t clock = 0;
};

std::mutex g_mu;
std::map<int, DeviceGraphs> g_dev;
int64_t g_counts[3] = {0, 0, 0};   // replays as recorded, updates in place, instantiations

// The graph's previous replay must have ended before its parameters change
// or it is destroyed.
hipError_t settle(GraphEntry& g) { return g.done ? hipEventSynchronize(g.done) : hipSuccess; }

void drop(GraphEntry& g) {
    settle(g);
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.done) hipEventDestroy(g.done);
    g.exec = nullptr;
    g.done = nullptr;
}

}  // namespace

int graph_replay(const std::string& topo, const std::string& full, const std::function<int(void*)>& record,
                 void* stream, int* how) {
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev)) return (int)e;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceGraphs& D = g_dev[dev];
    if (!D.capture) {
        if (hipError_t e = hipStreamCreateWithFlags(&D.capture, hipStreamNonBlocking)) {
            D.capture = nullptr;
            return (int)e;
        }
    }
    const hipStream_t st = (hipStream_t)stream;
    GraphEntry* g = nullptr;
    for (auto& x : D.entries)
        if (x.topo == topo) g = &x;
    auto launch = [&](GraphEntry& x) -> int {
        x.used = ++D.clock;
        if (hipError_t e = hipGraphLaunch(x.exec, st)) return (int)e;
        return (int)hipEventRecord(x.done, st);
    };
    if (g && g->full == full) {
        ++g_counts[0];
        if (how) *how = 0;
        return launch(*g);
    }
    // record the sequence with the new arguments
    if (hipError_t e = hipStreamBeginCapture(D.capture, hipStreamCaptureModeRelaxed)) return (int)e;
    const int rc = record(D.capture);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(D.capture, &graph);
    if (rc || ec) {
        if (graph) hipGraphDestroy(graph);
        return rc ? rc : (int)ec;
    }
    int err = 0;
    if (g) {
        // same topology: update the instantiated graph in place
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
        if (hipError_t e = settle(*g)) err = (int)e;
        if (!err && hipGraphExecUpdate(g->exec, graph, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            g->full = full;
            ++g_counts[1];
            if (how) *how = 1;
        } else if (!err) {
            (void)hipGetLastError();   // the refused update leaves an error behind
            drop(*g);
            g->topo.clear();
            g = nullptr;
        }
    }
    if (!err && !g) {
        // a free entry, else a new one, else the least recently used
        for (auto& x : D.entries)
            if (!g && !x.exec) g = &x;
        if (!g && (int)D.entries.size() < kGraphsPerDevice) {
            D.entries.emplace_back();
            g = &D.entries.back();
        }
        if (!g) {
            g = &D.entries[0];
            for (auto& x : D.entries)
                if (x.used < g->used) g = &x;
            drop(*g);
        }
        g->topo = topo;
        g->full = full;
        hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            drop(*g);
            g->topo.clear();
            g->full.clear();
            err = (int)e;
        } else {
            ++g_counts[2];
            if (how) *how = 2;
        }
    }
    hipGraphDestroy(graph);
    if (err) return err;
    return launch(*g);
}

void graph_counts(int64_t out[3]) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < 3; ++i) out[i] = g_counts[i];
}

void graph_key_add(std::string& key, const void* p, size_t n) { key.append(static_cast<const char*>(p), n); }

}  // namespace rx
