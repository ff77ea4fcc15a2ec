// Autotuner: successive halving over kernel variants and launch shapes.
//
// Every candidate runs the same lockstep machine, so every candidate must
// return the same bits (Thm. 7.2: the result of the parallel machine does not
// depend on the schedule); the tuner checks that on each candidate's first
// run and fails loudly on a disagreement.  Times are device times from HIP
// events on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "rx_internal.h"

namespace rx {

namespace {

struct Cand {
    rx_launch launch{};
    rx_multi_config multi{};
    double total_ms = 0;
    int runs = 0;
    double mean() const { return runs ? total_ms / runs : 1e30; }
};

template <class Run>
int halving(std::vector<Cand>& cands, int budget_runs, const uint8_t* d_out, size_t out_bytes, void* stream,
            Run run, int* best_index) {
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(RX_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(RX_EHIP, "hipEventCreate failed");
    }
    std::vector<uint8_t> ref, cur;
    int rc = RX_OK;
    std::vector<int> alive(cands.size());
    for (size_t i = 0; i < cands.size(); ++i) alive[i] = (int)i;
    int spent = 0;
    int reps = 1;
    while (rc == RX_OK && !alive.empty()) {
        for (int idx : alive) {
            Cand& c = cands[idx];
            for (int r = 0; r < reps && rc == RX_OK; ++r) {
                hipEventRecord(e0, st);
                if ((rc = run(c))) break;
                hipEventRecord(e1, st);
                if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(RX_EHIP, "hipEventSynchronize failed"); break; }
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (c.runs == 0) {
                    // determinacy: every candidate returns the first candidate's bits
                    cur.resize(out_bytes);
                    if (out_bytes && hipMemcpy(cur.data(), d_out, out_bytes, hipMemcpyDeviceToHost) != hipSuccess) {
                        rc = fail(RX_EHIP, "hipMemcpy of tuning results failed");
                        break;
                    }
                    if (ref.empty()) ref = cur;
                    else if (ref != cur) {
                        rc = fail(RX_EINVAL, "autotune: a candidate launch returned different bits (variant " +
                                                 std::to_string(c.launch.variant) + ", block " +
                                                 std::to_string(c.launch.block ? c.launch.block : c.multi.block) + ")");
                        break;
                    }
                    if (c.runs == 0 && r == 0 && reps == 1) {
                        // the first run also warms caches: time it again
                        hipEventRecord(e0, st);
                        if ((rc = run(c))) break;
                        hipEventRecord(e1, st);
                        hipEventSynchronize(e1);
                        hipEventElapsedTime(&ms, e0, e1);
                    }
                }
                c.total_ms += ms;
                c.runs += 1;
                ++spent;
            }
            if (rc) break;
        }
        if (rc || alive.size() == 1 || spent >= budget_runs) break;
        std::sort(alive.begin(), alive.end(), [&](int a, int b) { return cands[a].mean() < cands[b].mean(); });
        alive.resize((alive.size() + 1) / 2);
        reps *= 2;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    int best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (cands[i].runs && cands[i].mean() < cands[best].mean()) best = (int)i;
    *best_index = best;
    return RX_OK;
}

}  // namespace

int autotune_single(const Program* P, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t length, int64_t n,
                    uint8_t* d_out, int budget_runs, rx_launch* best, double* best_ms, int* n_cands, void* stream) {
    int cus = 256;
    if (hip_cu_count(&cus) || cus <= 0) cus = 256;
    std::vector<Cand> cands;
    auto add = [&](int v, int block, int grid) {
        Cand c;
        c.launch.variant = v;
        c.launch.block = block;
        c.launch.grid = grid;
        cands.push_back(c);
    };
    const bool fixed = d_offsets == nullptr;
    if (fixed && jit_ready(P, nullptr, nullptr) && length > 0 && length % 16 == 0 &&
        (reinterpret_cast<uintptr_t>(d_bytes) & 15) == 0)
        for (int burst : {1, 2, 3, 4, 5}) {
            add(RX_VARIANT_SLICED, 0, 0);
            cands.back().launch.unroll = burst;
        }
    if (P->W <= kLaneMaxWords)
        for (int block : {64, 128, 256})
            for (int gm : {0, 2, 4, 8}) add(RX_VARIANT_LANE, block, gm * cus);
    for (int block : {64, 256, 1024})
        for (int gm : {0, 4}) add(RX_VARIANT_WAVE, block, gm * cus);
    // lanes per set: 64 (one wavefront per string) up to 1024 (sixteen wavefronts per string)
    for (int ws : {2, 4, 8, 16}) {
        add(RX_VARIANT_WAVE, 0, 0);
        cands.back().launch.unroll = ws;
    }
    if (n_cands) *n_cands = (int)cands.size();
    auto run = [&](const Cand& c) -> int {
        return fixed ? rx_match_fixed_ex(reinterpret_cast<const rx_program*>(P), d_bytes, length, n, d_out, &c.launch, stream)
                     : rx_match_ex(reinterpret_cast<const rx_program*>(P), d_bytes, d_offsets, n, d_out, &c.launch, stream);
    };
    int bi = 0;
    if (int rc = halving(cands, budget_runs, d_out, (size_t)n, stream, run, &bi)) return rc;
    *best = cands[bi].launch;
    if (best_ms) *best_ms = cands[bi].mean();
    return RX_OK;
}

int autotune_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes, const int64_t* d_offsets,
                   int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes, int budget_runs, rx_multi_config* best,
                   double* best_ms, int* n_cands, void* stream) {
    int cus = 256;
    if (hip_cu_count(&cus) || cus <= 0) cus = 256;
    std::vector<std::vector<int>> ladders;
    {
        std::vector<int> pow2, fine, coarse;
        for (int e = 8; e <= 4096; e *= 2) pow2.push_back(e);
        for (double e = 8; e <= 4096 && fine.size() < 15; e *= 1.56) fine.push_back((int)e);
        coarse = {16, 128, 1024};
        ladders = {pow2, fine, coarse};
    }
    std::vector<Cand> cands;
    for (const auto& lad : ladders)
        for (int block : {64, 128, 256})
            for (int gm : {2, 4, 8}) {
                Cand c;
                c.multi.n_edges = (int)lad.size();
                for (size_t i = 0; i < lad.size(); ++i) c.multi.edges[i] = lad[i];
                c.multi.block = block;
                c.multi.grid = gm * cus;
                cands.push_back(c);
            }
    // the plane form (bit-sliced circuits), when the list has its module and the workspace holds the planes
    if (n > 0) {
        std::vector<const Program*> ps(n_progs);
        for (int i = 0; i < n_progs; ++i) ps[i] = reinterpret_cast<const Program*>(progs[i]);
        int64_t ends[2] = {0, 0};
        if (jit_planes_prepared(ps.data(), n_progs) &&
            hipMemcpy(&ends[0], d_offsets, 8, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(&ends[1], d_offsets + n, 8, hipMemcpyDeviceToHost) == hipSuccess) {
            const int64_t total = ends[1] - ends[0];
            if (total >= 0 && plane_workspace_bytes(n, total, n_progs, 256) <= (int64_t)work_bytes) {
                Cand c;
                c.multi.form = RX_FORM_PLANES;
                c.multi.max_bytes = total;
                cands.push_back(c);
            }
        }
    }
    if (n_cands) *n_cands = (int)cands.size();
    auto run = [&](const Cand& c) -> int {
        return rx_match_multi(progs, n_progs, d_bytes, d_offsets, n, d_out, d_work, work_bytes, &c.multi, stream);
    };
    int bi = 0;
    if (int rc = halving(cands, budget_runs, d_out, (size_t)n * (size_t)n_progs, stream, run, &bi)) return rc;
    *best = cands[bi].multi;
    if (best_ms) *best_ms = cands[bi].mean();
    return RX_OK;
}

}  // namespace rx
