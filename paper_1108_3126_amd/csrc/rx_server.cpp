// Serving loop: continuous batching of match requests.
//
// Clients submit requests (an expression plus a batch of host strings) from
// any thread.  A scheduler thread admits pending requests into the next free
// step slot while they fit its device capacity (strings, bytes, requests,
// distinct programs), so the total device memory the server holds -- every
// slot plus the resident program tables -- stays inside the configured HBM
// budget.  Requests that arrive while steps run join the next step; with two
// or more slots, steps overlap on the device on separate streams.  A step is
// one work-item launch (the persistent item kernel of the batched matcher)
// framed by three host-to-device copies and one copy back, replayed as a
// hipGraph whose node parameters are updated per step.  Compiled programs
// stay resident in a device arena keyed by the request's expression, with
// least-recently-used eviction of tables no running step reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rx_internal.h"

namespace rx {

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kArenaSlotBytes = 64 * 1024;  // one program's tables (sets of at most 16 words)
constexpr int64_t kItemHeader = 256;            // queue header (item count, head) before the items

struct CacheEntry {
    Program* prog = nullptr;
    int arena_slot = -1;
    int inflight = 0;          // running steps that read these tables
    uint64_t last_used = 0;
    int upload_slot = -1;      // the slot whose stream carried the last upload of the tables
    uint64_t upload_seq = 0;   // the step of that slot which enqueued it
};

struct Request {
    int64_t id = 0;
    CacheEntry* entry = nullptr;
    std::vector<uint8_t> bytes;
    std::vector<int64_t> offsets;  // rebased to start at 0
    int64_t n = 0;
    std::vector<uint8_t> result;
    Clock::time_point t_submit, t_done;
    bool done = false;
    int status = RX_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    hipEvent_t start_ev = nullptr;
    hipEvent_t upload_ev = nullptr;   // after the program uploads of the slot's current step
    uint64_t seq = 0;                 // the step the slot is running
    bool uploaded = false;            // the current step enqueued uploads
    uint8_t *h_bytes = nullptr, *h_out = nullptr, *h_items = nullptr;
    int64_t* h_offs = nullptr;
    uint8_t *d_bytes = nullptr, *d_out = nullptr, *d_items = nullptr;
    int64_t* d_offs = nullptr;
    std::vector<Request*> reqs;
    std::vector<int64_t> line0;
    std::vector<CacheEntry*> entries;
    bool busy = false;
    StepGraph* graph = nullptr;
};

}  // namespace

struct Server {
    rx_server_config cfg{};
    int dev = 0;
    int64_t max_items = 0;
    uint8_t* d_arena = nullptr;
    std::vector<CacheEntry*> arena_owner;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<int64_t, Request*> requests;
    std::unordered_map<std::string, CacheEntry*> cache;
    std::thread worker;
    std::atomic<bool> stop{false};
    int fatal = RX_OK;
    std::string fatal_msg;
    int64_t next_id = 1;
    uint64_t step_seq = 0;
    // statistics
    std::vector<double> lat_us;
    int64_t submitted = 0, completed = 0, rejected = 0, steps = 0, graph_steps = 0, strings = 0, bytes = 0;
    int64_t hits = 0, misses = 0, evictions = 0, max_queue = 0;
    double pack_ms = 0, device_ms = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;

    ~Server();
    int init();
    void run();
    bool launch_step(Slot& s, std::vector<Request*>& take);
    void complete(Slot& s);
    int ensure_resident(CacheEntry* e, Slot& s);
    void fail_pending_locked(int rc);
    int max_step_programs() const;
};

static int hip_err(hipError_t e, const char* what) {
    return fail(RX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int Server::init() {
    if (hipGetDevice(&dev) != hipSuccess) return fail(RX_EHIP, "hipGetDevice failed");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (cfg.grid <= 0) cfg.grid = 4 * cus;
    max_items = cfg.step_strings / cfg.block + cfg.step_requests + 1;
    arena_owner.assign(cfg.program_slots, nullptr);
    if (hipError_t e = hipMalloc(&d_arena, (size_t)cfg.program_slots * kArenaSlotBytes)) return hip_err(e, "hipMalloc arena");
    slots.resize(cfg.slots);
    for (Slot& s : slots) {
        const size_t nb = (size_t)cfg.step_bytes + 16, no = 8 * (size_t)(cfg.step_strings + 1),
                     ni = kItemHeader + sizeof(WorkItem) * (size_t)max_items, nr = (size_t)cfg.step_strings;
        hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (!e) e = hipEventCreate(&s.done_ev);
        if (!e) e = hipEventCreate(&s.start_ev);
        if (!e) e = hipEventCreateWithFlags(&s.upload_ev, hipEventDisableTiming);
        if (!e) e = hipHostMalloc((void**)&s.h_bytes, nb, hipHostMallocDefault);
        if (!e) e = hipHostMalloc((void**)&s.h_offs, no, hipHostMallocDefault);
        if (!e) e = hipHostMalloc((void**)&s.h_items, ni, hipHostMallocDefault);
        if (!e) e = hipHostMalloc((void**)&s.h_out, nr, hipHostMallocDefault);
        if (!e) e = hipMalloc(&s.d_bytes, nb);
        if (!e) e = hipMalloc(&s.d_offs, no);
        if (!e) e = hipMalloc(&s.d_items, ni);
        if (!e) e = hipMalloc(&s.d_out, nr);
        if (e) return hip_err(e, "server buffers");
    }
    worker = std::thread([this] { run(); });
    return RX_OK;
}

Server::~Server() {
    stop = true;
    cv_submit.notify_all();
    if (worker.joinable()) worker.join();
    for (Slot& s : slots) {
        if (s.stream) hipStreamSynchronize(s.stream);
        step_graph_destroy(s.graph);
        if (s.done_ev) hipEventDestroy(s.done_ev);
        if (s.start_ev) hipEventDestroy(s.start_ev);
        if (s.upload_ev) hipEventDestroy(s.upload_ev);
        if (s.stream) hipStreamDestroy(s.stream);
        hipHostFree(s.h_bytes);
        hipHostFree(s.h_offs);
        hipHostFree(s.h_items);
        hipHostFree(s.h_out);
        hipFree(s.d_bytes);
        hipFree(s.d_offs);
        hipFree(s.d_items);
        hipFree(s.d_out);
    }
    if (d_arena) hipFree(d_arena);
    for (auto& kv : cache) {
        jit_free(kv.second->prog);
        delete kv.second->prog;
        delete kv.second;
    }
    for (auto& kv : requests) delete kv.second;
}

// Places the entry's tables in a device arena slot (evicting the least
// recently used entry no running step reads); the copy is ordered on `s`.
int Server::ensure_resident(CacheEntry* e, Slot& s) {
    TraceRange trace_range_("rx_server.resident");
    if (e->arena_slot >= 0) {
        ++hits;
        return RX_OK;
    }
    ++misses;
    int victim = -1;
    uint64_t oldest = ~0ull;
    for (int i = 0; i < (int)arena_owner.size(); ++i) {
        CacheEntry* o = arena_owner[i];
        if (!o) { victim = i; break; }
        if (o->inflight == 0 && o->last_used < oldest) { oldest = o->last_used; victim = i; }
    }
    if (victim < 0) return fail(RX_EBUSY, "every resident program is in use");
    if (arena_owner[victim]) {
        arena_owner[victim]->arena_slot = -1;
        ++evictions;
    }
    arena_owner[victim] = e;
    e->arena_slot = victim;
    uint8_t* dst = d_arena + (int64_t)victim * kArenaSlotBytes;
    if (hipError_t err = hipMemcpyAsync(dst, e->prog->blob.data(), e->prog->blob.size(), hipMemcpyHostToDevice, s.stream))
        return hip_err(err, "program upload");
    e->upload_slot = (int)(&s - slots.data());
    e->upload_seq = step_seq;
    s.uploaded = true;
    return RX_OK;
}

// Distinct programs one step may use.  With every slot's step holding at most
// this many arena entries, a step being assembled always finds an entry no
// running step reads, so ensure_resident never runs out of slots.
int Server::max_step_programs() const {
    const int per_slot = cfg.program_slots / std::max(1, cfg.slots);
    return std::max(1, std::min(kMaxItemProgs, per_slot));
}

// Fails every request still waiting for a step (the server has stopped or a
// step failed); their waiters wake up with the status.  Caller holds mu.
void Server::fail_pending_locked(int rc) {
    const Clock::time_point now = Clock::now();
    for (Request* r : pending) {
        r->status = rc;
        r->done = true;
        r->t_done = now;
    }
    pending.clear();
    cv_done.notify_all();
}

bool Server::launch_step(Slot& s, std::vector<Request*>& take) {
    TraceRange trace_range_("rx_server.step");
    const Clock::time_point t0 = Clock::now();
    ++step_seq;
    s.seq = step_seq;
    s.uploaded = false;
    hipEventRecord(s.start_ev, s.stream);
    s.reqs = take;
    s.line0.clear();
    s.entries.clear();
    std::vector<CacheEntry*> progs;
    StepDesc d{};
    int64_t line = 0, byte = 0, items = 0;
    WorkItem* it = reinterpret_cast<WorkItem*>(s.h_items + kItemHeader);
    int rc = RX_OK;
    for (Request* r : take) {
        int pidx = -1;
        for (size_t i = 0; i < progs.size(); ++i)
            if (progs[i] == r->entry) pidx = (int)i;
        if (pidx < 0) {
            if ((rc = ensure_resident(r->entry, s))) break;
            pidx = (int)progs.size();
            progs.push_back(r->entry);
            const Program* P = r->entry->prog;
            const uint8_t* base = d_arena + (int64_t)r->entry->arena_slot * kArenaSlotBytes;
            ProgDesc& pd = d.items.progs[pidx];
            pd.first = reinterpret_cast<const uint32_t*>(base + P->layout.first);
            pd.follow = reinterpret_cast<const uint32_t*>(base + P->layout.follow);
            pd.bytemask = reinterpret_cast<const uint32_t*>(base + P->layout.bytemask);
            pd.L = P->L;
            pd.W = P->W;
            pd.suffix_any = P->suffix_any ? 1 : 0;
            pd.pad = 0;
        }
        r->entry->inflight += 1;
        r->entry->last_used = step_seq;
        s.entries.push_back(r->entry);
        // tables uploaded by a step still running on another slot: this step's
        // stream waits for that upload (it was enqueued on the other stream)
        const int us = r->entry->upload_slot;
        if (pidx == (int)progs.size() - 1 && us >= 0 && &slots[us] != &s && slots[us].busy &&
            slots[us].seq == r->entry->upload_seq) {
            if (hipError_t e = hipStreamWaitEvent(s.stream, slots[us].upload_ev, 0)) {
                rc = hip_err(e, "wait for a program upload");
                break;
            }
        }
        if (!r->bytes.empty()) std::memcpy(s.h_bytes + byte, r->bytes.data(), r->bytes.size());
        for (int64_t i = 0; i < r->n; ++i) s.h_offs[line + i] = r->offsets[i] + byte;
        for (int64_t t = 0; t < r->n; t += cfg.block) {
            WorkItem w;
            w.prog = pidx;
            w.count = (int32_t)std::min<int64_t>(cfg.block, r->n - t);
            w.line0 = line + t;
            w.out0 = 0;
            it[items++] = w;
        }
        s.line0.push_back(line);
        line += r->n;
        byte += (int64_t)r->bytes.size();
    }
    s.h_offs[line] = byte;
    if (rc == RX_OK && s.uploaded)
        if (hipError_t e = hipEventRecord(s.upload_ev, s.stream)) rc = hip_err(e, "record the program uploads");
    reinterpret_cast<int32_t*>(s.h_items)[0] = (int32_t)items;  // item count
    reinterpret_cast<int32_t*>(s.h_items)[1] = 0;               // queue head
    if (rc == RX_OK) {
        d.h2d[0] = {s.d_bytes, s.h_bytes, (size_t)byte};
        d.h2d[1] = {s.d_offs, s.h_offs, 8 * (size_t)(line + 1)};
        d.h2d[2] = {s.d_items, s.h_items, (size_t)(kItemHeader + sizeof(WorkItem) * items)};
        d.items.n_progs = (int32_t)progs.size();
        d.items.block = cfg.block;
        d.items.grid = cfg.grid;
        d.items.bytes = s.d_bytes;
        d.items.offsets = s.d_offs;
        d.items.items = reinterpret_cast<const WorkItem*>(s.d_items + kItemHeader);
        d.items.n_items = reinterpret_cast<const int32_t*>(s.d_items);
        d.items.head = reinterpret_cast<int32_t*>(s.d_items) + 1;
        d.items.out = s.d_out;
        d.items.stream = s.stream;
        d.d2h = {s.h_out, s.d_out, (size_t)line};
        int e;
        if (cfg.use_graph) {
            e = step_graph_launch(&s.graph, d, s.stream);
            if (e == 0) ++graph_steps;
        } else {
            e = step_launch_direct(d, s.stream);
        }
        if (e == 0) e = (int)hipEventRecord(s.done_ev, s.stream);
        if (e) rc = fail(RX_EHIP, std::string("serving step: ") + hip_error_string(e));
    }
    if (rc != RX_OK) {
        std::lock_guard<std::mutex> g(mu);
        for (CacheEntry* e : s.entries) e->inflight -= 1;
        for (Request* r : take) {
            r->status = rc;
            r->done = true;
            r->t_done = Clock::now();
        }
        s.reqs.clear();
        s.entries.clear();
        fatal = rc;
        fatal_msg = last_error_cstr();
        fail_pending_locked(rc);
        return false;
    }
    s.busy = true;
    ++steps;
    pack_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    return true;
}

void Server::complete(Slot& s) {
    TraceRange trace_range_("rx_server.complete");
    const Clock::time_point now = Clock::now();
    float dev_ms = 0;
    hipEventElapsedTime(&dev_ms, s.start_ev, s.done_ev);
    std::lock_guard<std::mutex> g(mu);
    device_ms += dev_ms;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        Request* r = s.reqs[i];
        r->result.assign(s.h_out + s.line0[i], s.h_out + s.line0[i] + r->n);
        r->done = true;
        r->t_done = now;
        lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        ++completed;
        strings += r->n;
        bytes += (int64_t)r->bytes.size();
        std::vector<uint8_t>().swap(r->bytes);
        std::vector<int64_t>().swap(r->offsets);
    }
    for (CacheEntry* e : s.entries) e->inflight -= 1;
    t_last = now;
    s.reqs.clear();
    s.entries.clear();
    s.busy = false;
    cv_done.notify_all();
}

void Server::run() {
    if (hipSetDevice(dev) != hipSuccess) return;
    while (true) {
        for (Slot& s : slots)
            if (s.busy && hipEventQuery(s.done_ev) == hipSuccess) complete(s);
        Slot* free_slot = nullptr;
        for (Slot& s : slots)
            if (!s.busy) { free_slot = &s; break; }
        std::vector<Request*> take;
        {
            std::unique_lock<std::mutex> lk(mu);
            // after a failed step nothing more runs: waiting requests fail at once
            if (fatal != RX_OK && !pending.empty()) fail_pending_locked(fatal);
            // on destruction, pending requests still run (drain) unless a step has failed
            if (stop && pending.empty()) {
                bool any_busy = false;
                for (Slot& s : slots) any_busy |= s.busy;
                if (!any_busy) break;
            }
            if (free_slot && !pending.empty() && fatal == RX_OK) {
                int64_t nb = 0, ns = 0;
                std::vector<CacheEntry*> distinct;
                while (!pending.empty()) {
                    Request* r = pending.front();
                    const bool fresh = std::find(distinct.begin(), distinct.end(), r->entry) == distinct.end();
                    if ((int)take.size() >= cfg.step_requests || ns + r->n > cfg.step_strings ||
                        nb + (int64_t)r->bytes.size() > cfg.step_bytes ||
                        (fresh && (int)distinct.size() >= max_step_programs()))
                        break;
                    if (fresh) distinct.push_back(r->entry);
                    take.push_back(r);
                    ns += r->n;
                    nb += (int64_t)r->bytes.size();
                    pending.pop_front();
                }
            } else if (!free_slot) {
                // every slot busy: fall through to wait on the oldest step
            } else {
                cv_submit.wait_for(lk, std::chrono::microseconds(100));
                continue;
            }
        }
        if (!take.empty()) {
            // arena, cache-entry residency and step state are touched only by this thread
            launch_step(*free_slot, take);
            continue;
        }
        if (!free_slot) {
            for (Slot& s : slots)
                if (s.busy) {
                    hipEventSynchronize(s.done_ev);
                    complete(s);
                    break;
                }
        }
    }
}

}  // namespace rx

using namespace rx;

extern "C" {

int rx_server_create(const rx_server_config* cfg_in, rx_server** out) {
    try {
        if (!out) return fail(RX_EINVAL, "out is NULL");
        *out = nullptr;
        rx_server_config c{};
        if (cfg_in) c = *cfg_in;
        if (c.step_bytes <= 0) c.step_bytes = 64ll << 20;
        if (c.step_strings <= 0) c.step_strings = 1 << 18;
        if (c.step_requests <= 0) c.step_requests = 512;
        if (c.slots <= 0) c.slots = 2;
        if (c.block <= 0) c.block = 256;
        if (c.program_slots <= 0) c.program_slots = 1024;
        if (c.hbm_budget <= 0) c.hbm_budget = 2ll << 30;
        if (c.block != 64 && c.block != 128 && c.block != 256) return fail(RX_EINVAL, "block must be 64, 128 or 256");
        if (c.slots > 8) return fail(RX_EINVAL, "at most 8 slots");
        if (c.program_slots < c.slots) return fail(RX_EINVAL, "program_slots must be at least slots");
        const int64_t max_items = c.step_strings / c.block + c.step_requests + 1;
        const int64_t per_slot = (c.step_bytes + 16) + 8 * (c.step_strings + 1) + kItemHeader +
                                 (int64_t)sizeof(WorkItem) * max_items + c.step_strings;
        const int64_t need = c.slots * per_slot + (int64_t)c.program_slots * kArenaSlotBytes;
        if (need > c.hbm_budget)
            return fail(RX_ETOOBIG, "slots and program arena need " + std::to_string(need) +
                                        " device bytes; the budget is " + std::to_string(c.hbm_budget));
        Server* S = new Server;
        S->cfg = c;
        if (int rc = S->init()) {
            const std::string msg = last_error_cstr();
            delete S;
            return fail(rc, msg);
        }
        *out = reinterpret_cast<rx_server*>(S);
        return RX_OK;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}

void rx_server_destroy(rx_server* srv) {
    try {
        delete reinterpret_cast<Server*>(srv);
    } catch (...) {
    }
}

int rx_server_submit(rx_server* srv, const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
                     int32_t n_classes, uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets,
                     int64_t n, int64_t* req_id) {
    try {
        Server* S = reinterpret_cast<Server*>(srv);
        if (!S || !req_id) return fail(RX_EINVAL, "NULL argument");
        if (n < 0 || (n > 0 && !host_offsets)) return fail(RX_EINVAL, "bad string batch");
        const int64_t base = n > 0 ? host_offsets[0] : 0;
        const int64_t nbytes = n > 0 ? host_offsets[n] - base : 0;
        for (int64_t i = 0; i < n; ++i)
            if (host_offsets[i + 1] < host_offsets[i]) return fail(RX_EINVAL, "offsets must not decrease");
        if (nbytes > 0 && !host_bytes) return fail(RX_EINVAL, "bytes is NULL");
        if (n > S->cfg.step_strings || nbytes > S->cfg.step_bytes)
            return fail(RX_ETOOBIG, "request exceeds one step's capacity (" + std::to_string(S->cfg.step_strings) +
                                        " strings, " + std::to_string(S->cfg.step_bytes) + " bytes)");
        std::string key;
        key.append(reinterpret_cast<const char*>(&n_ast), sizeof(n_ast));
        key.append(reinterpret_cast<const char*>(&root), sizeof(root));
        key.append(reinterpret_cast<const char*>(&flags), sizeof(flags));
        if (ast && n_ast > 0) key.append(reinterpret_cast<const char*>(ast), sizeof(rx_ast_node) * (size_t)n_ast);
        if (classes && n_classes > 0) key.append(reinterpret_cast<const char*>(classes), sizeof(rx_class) * (size_t)n_classes);
        Request* r = new Request;
        r->n = n;
        r->t_submit = Clock::now();
        if (nbytes > 0) r->bytes.assign(host_bytes + base, host_bytes + base + nbytes);
        r->offsets.resize(n + 1);
        for (int64_t i = 0; i <= n; ++i) r->offsets[i] = n > 0 ? host_offsets[i] - base : 0;
        CacheEntry* entry = nullptr;
        {
            std::lock_guard<std::mutex> g(S->mu);
            if (S->fatal) {
                delete r;
                return fail(S->fatal, "server failed: " + S->fatal_msg);
            }
            auto found = S->cache.find(key);
            if (found != S->cache.end()) entry = found->second;
        }
        if (!entry) {
            Program* P = nullptr;
            if (int rc = compile(ast, n_ast, root, classes, n_classes, flags, &P)) {
                delete r;
                std::lock_guard<std::mutex> g(S->mu);
                ++S->rejected;
                return rc;
            }
            if (P->W > kLaneMaxWords || P->blob.size() > (size_t)kArenaSlotBytes) {
                delete P;
                delete r;
                std::lock_guard<std::mutex> g(S->mu);
                ++S->rejected;
                return fail(RX_ETOOBIG, "the server holds programs with at most 511 leaves");
            }
            std::lock_guard<std::mutex> g(S->mu);
            auto found = S->cache.find(key);
            if (found != S->cache.end()) {
                delete P;
                entry = found->second;
            } else {
                entry = new CacheEntry;
                entry->prog = P;
                S->cache.emplace(key, entry);
            }
        }
        {
            std::lock_guard<std::mutex> g(S->mu);
            r->entry = entry;
            r->id = S->next_id++;
            S->requests.emplace(r->id, r);
            S->pending.push_back(r);
            ++S->submitted;
            if ((int64_t)S->pending.size() > S->max_queue) S->max_queue = (int64_t)S->pending.size();
            if (!S->have_first) {
                S->have_first = true;
                S->t_first = r->t_submit;
            }
            *req_id = r->id;
        }
        S->cv_submit.notify_one();
        return RX_OK;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}

int rx_server_wait(rx_server* srv, int64_t req_id, uint8_t* host_out, int64_t timeout_us) {
    try {
        Server* S = reinterpret_cast<Server*>(srv);
        if (!S) return fail(RX_EINVAL, "server is NULL");
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->requests.find(req_id);
        if (it == S->requests.end()) return fail(RX_EINVAL, "unknown request id");
        Request* r = it->second;
        auto ready = [&] { return r->done; };
        if (timeout_us < 0) S->cv_done.wait(lk, ready);
        else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return fail(RX_ETIMEOUT, "request not finished");
        const int status = r->status;
        if (status == RX_OK && host_out && r->n) std::memcpy(host_out, r->result.data(), (size_t)r->n);
        S->requests.erase(it);
        delete r;
        if (status != RX_OK) return fail(status, "request failed: " + S->fatal_msg);
        return RX_OK;
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}

int rx_server_stats(rx_server* srv, rx_server_counters* out) {
    Server* S = reinterpret_cast<Server*>(srv);
    if (!S || !out) return fail(RX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->steps = S->steps;
    out->graph_steps = S->graph_steps;
    out->strings = S->strings;
    out->bytes = S->bytes;
    out->cache_hits = S->hits;
    out->cache_misses = S->misses;
    out->cache_evictions = S->evictions;
    out->max_queue = S->max_queue;
    out->queued = (int64_t)S->pending.size();
    out->pack_ms = S->pack_ms;
    out->device_ms = S->device_ms;
    if (!S->lat_us.empty()) {
        std::vector<double> v = S->lat_us;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5))]; };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        double s = 0;
        for (double x : v) s += x;
        out->mean_us = s / (double)v.size();
        out->max_us = v.back();
    }
    if (S->have_first && S->completed)
        out->wall_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
    return RX_OK;
}

int rx_server_reset_stats(rx_server* srv) {
    Server* S = reinterpret_cast<Server*>(srv);
    if (!S) return fail(RX_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    S->lat_us.clear();
    S->submitted = S->completed = S->rejected = S->steps = S->graph_steps = S->strings = S->bytes = 0;
    S->hits = S->misses = S->evictions = S->max_queue = 0;
    S->pack_ms = S->device_ms = 0;
    S->have_first = false;
    return RX_OK;
}

// The per-request plain path: compile, upload, copy in, one launch, copy out,
// synchronise, free.  Used as the baseline the batched server is measured against.
int rx_plain_match(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes, int32_t n_classes,
                   uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets, int64_t n,
                   uint8_t* host_out) {
    try {
        if (n < 0 || (n > 0 && (!host_offsets || !host_out))) return fail(RX_EINVAL, "bad string batch");
        Program* P = nullptr;
        if (int rc = compile(ast, n_ast, root, classes, n_classes, flags, &P)) return rc;
        const int64_t base = n > 0 ? host_offsets[0] : 0;
        const int64_t nbytes = n > 0 ? host_offsets[n] - base : 0;
        std::vector<int64_t> offs(n + 1);
        for (int64_t i = 0; i <= n; ++i) offs[i] = n > 0 ? host_offsets[i] - base : 0;
        void *d_tab = nullptr, *d_bytes = nullptr, *d_offs = nullptr, *d_out = nullptr;
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (!e) e = hipMalloc(&d_tab, P->blob.size());
        if (!e) e = hipMalloc(&d_bytes, (size_t)nbytes + 16);
        if (!e) e = hipMalloc(&d_offs, 8 * (size_t)(n + 1));
        if (!e) e = hipMalloc(&d_out, (size_t)n + 1);
        int rc = RX_OK;
        if (!e) rc = rx_program_upload(reinterpret_cast<rx_program*>(P), d_tab, P->blob.size(), st);
        if (!e && !rc && nbytes) e = hipMemcpyAsync(d_bytes, host_bytes + base, (size_t)nbytes, hipMemcpyHostToDevice, st);
        if (!e && !rc) e = hipMemcpyAsync(d_offs, offs.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, st);
        if (!e && !rc && n)
            rc = rx_match(reinterpret_cast<const rx_program*>(P), static_cast<const uint8_t*>(d_bytes),
                          static_cast<const int64_t*>(d_offs), n, static_cast<uint8_t*>(d_out), st);
        if (!e && !rc && n) e = hipMemcpyAsync(host_out, d_out, (size_t)n, hipMemcpyDeviceToHost, st);
        if (!e && !rc) e = hipStreamSynchronize(st);
        if (st) {
            hipStreamSynchronize(st);
            hipStreamDestroy(st);
        }
        hipFree(d_tab);
        hipFree(d_bytes);
        hipFree(d_offs);
        hipFree(d_out);
        delete P;
        if (e) return hip_err(e, "plain match");
        return rc;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}

// The plain path with its resources made once: one stream and device buffers
// sized for the largest request, reused by every call.  Per request it does
// exactly compile, upload, copy in, one launch, copy out, synchronise.
struct rx_plain {
    hipStream_t stream = nullptr;
    void* d_tab = nullptr;
    size_t tab_cap = 0;
    void* d_bytes = nullptr;
    void* d_offs = nullptr;
    void* d_out = nullptr;
    int64_t max_bytes = 0, max_strings = 0;
    std::vector<int64_t> offs;
};

int rx_plain_create(int64_t max_bytes, int64_t max_strings, rx_plain** out) {
    try {
        if (!out || max_bytes < 0 || max_strings < 0) return fail(RX_EINVAL, "bad argument");
        *out = nullptr;
        rx_plain* c = new rx_plain;
        c->max_bytes = max_bytes;
        c->max_strings = max_strings;
        c->tab_cap = 1 << 20;
        c->offs.resize((size_t)max_strings + 1);
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (!e) e = hipMalloc(&c->d_tab, c->tab_cap);
        if (!e) e = hipMalloc(&c->d_bytes, (size_t)max_bytes + 16);
        if (!e) e = hipMalloc(&c->d_offs, 8 * (size_t)(max_strings + 1));
        if (!e) e = hipMalloc(&c->d_out, (size_t)max_strings + 1);
        if (e) {
            rx_plain_destroy(c);
            return hip_err(e, "plain path buffers");
        }
        *out = c;
        return RX_OK;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    }
}

void rx_plain_destroy(rx_plain* c) {
    if (!c) return;
    if (c->stream) {
        hipStreamSynchronize(c->stream);
        hipStreamDestroy(c->stream);
    }
    hipFree(c->d_tab);
    hipFree(c->d_bytes);
    hipFree(c->d_offs);
    hipFree(c->d_out);
    delete c;
}

int rx_plain_run(rx_plain* c, const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
                 int32_t n_classes, uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets, int64_t n,
                 uint8_t* host_out) {
    try {
        if (!c) return fail(RX_EINVAL, "context is NULL");
        if (n < 0 || (n > 0 && (!host_offsets || !host_out))) return fail(RX_EINVAL, "bad string batch");
        const int64_t base = n > 0 ? host_offsets[0] : 0;
        const int64_t nbytes = n > 0 ? host_offsets[n] - base : 0;
        if (n > c->max_strings || nbytes > c->max_bytes)
            return fail(RX_ETOOBIG, "request above the context's capacity");
        if (nbytes > 0 && !host_bytes) return fail(RX_EINVAL, "bytes is NULL");
        Program* P = nullptr;
        if (int rc = compile(ast, n_ast, root, classes, n_classes, flags, &P)) return rc;
        std::unique_ptr<Program> hold(P);
        if (P->blob.size() > c->tab_cap)
            return fail(RX_ETOOBIG, "program tables above the context's table buffer");
        for (int64_t i = 0; i <= n; ++i) c->offs[i] = n > 0 ? host_offsets[i] - base : 0;
        int rc = rx_program_upload(reinterpret_cast<rx_program*>(P), c->d_tab, c->tab_cap, c->stream);
        hipError_t e = hipSuccess;
        if (!rc && nbytes) e = hipMemcpyAsync(c->d_bytes, host_bytes + base, (size_t)nbytes, hipMemcpyHostToDevice,
                                              c->stream);
        if (!rc && !e) e = hipMemcpyAsync(c->d_offs, c->offs.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice,
                                          c->stream);
        if (!rc && !e && n)
            rc = rx_match(reinterpret_cast<const rx_program*>(P), static_cast<const uint8_t*>(c->d_bytes),
                          static_cast<const int64_t*>(c->d_offs), n, static_cast<uint8_t*>(c->d_out), c->stream);
        if (!rc && !e && n) e = hipMemcpyAsync(host_out, c->d_out, (size_t)n, hipMemcpyDeviceToHost, c->stream);
        const hipError_t es = hipStreamSynchronize(c->stream);
        if (!e) e = es;
        if (e) return hip_err(e, "plain match");
        return rc;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}

}  // extern "C"
