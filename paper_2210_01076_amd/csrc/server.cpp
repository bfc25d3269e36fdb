// Serving: many sessions resident on one device, updated by a stream of
// modify+update requests with continuous batching.
//
//  - Admission: a session holds device memory (state, checkpoints, plans and
//    scratch) only while resident.  A request's edits are applied and its
//    update planned on the host first; the session is then charged the
//    bytes it will hold after that update (which may have grown: added
//    levels add checkpoints) and admitted when they fit the budget, evicting
//    idle sessions (least recently used first) when needed.  A request that
//    cannot be admitted yet waits; one that can never fit fails with
//    QTASK_E_NOMEM and its edits are undone.
//  - Large sessions (n >= small_qubits) replay on their own streams (default
//    priority), up to max_inflight at once, so their passes overlap on the
//    device.
//  - Small sessions are batched: every tick, pass i of each ready small
//    session goes into one launch of the batched pass kernel (items found by
//    binary search over their first workgroup), followed by one launch that
//    sums their renormalisation partials.  The item tables live in device
//    memory at fixed addresses, so a fixed sequence of rounds is captured
//    once in a HIP graph and replayed with new tables each tick.
//  - Requests that arrive while a tick or a large update runs join the next
//    tick (continuous batching); every result carries submit/start/done
//    stamps and the state hash.
//  - Waiting requests start oldest first, or (order 1) expected-shortest
//    first, the estimate 2^n x levels divided by 1 + waiting time / 1 s.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "../../include/qtask.h"
#include "device.h"
#include "lowering.h"
#include "session.h"

using qtask::now_ms;
using qtask::Session;

namespace qtask {
Session *session_of(qtask_t h);
void set_server_owned(qtask_t h, bool owned);
}  // namespace qtask

namespace {

constexpr uint32_t kMaxItems = 256;        // sessions per batched round
constexpr uint32_t kRoundCaps[] = {8, 32, 128};
constexpr uint32_t kGroupCaps[] = {256, 2048, 16384};

struct Request {
    uint64_t ticket = 0;
    int32_t sid = 0;
    std::vector<qtask_edit> edits;
    double submit_ms = 0;
};

// waiting time that halves a request's expected-cost key under order 1
constexpr double kAgingMs = 1000.0;

struct SSession {
    Session *s = nullptr;
    qtask_t handle = nullptr;
    bool resident = false;
    bool busy = false;
    bool small = false;
    bool batched = false;   // current request runs in the batched ticks
    bool counted = false;   // current request holds a large-session slot
    bool waiting = false;   // current request is planned and waits for memory
    uint64_t bytes = 0;     // bytes charged to the budget while resident
    double last_used = 0;
    std::deque<Request> q;
    Request cur;
    double start_ms = 0;
    int status = QTASK_OK;
    hipEvent_t done = nullptr;
};

struct GraphKey {
    int dtype, mf, threads, rounds, groups;
    bool operator<(const GraphKey &o) const {
        return std::tie(dtype, mf, threads, rounds, groups) < std::tie(o.dtype, o.mf, o.threads, o.rounds, o.groups);
    }
};

struct BatchTables {
    KBatchItem *d_items = nullptr;   // [round][kMaxItems]
    uint32_t *d_counts = nullptr;    // [round] pass items, then [round] sum items
    KSumItem *d_sums = nullptr;      // [round][kMaxItems]
    KBatchItem *h_items = nullptr;   // pinned staging
    uint32_t *h_counts = nullptr;
    KSumItem *h_sums = nullptr;
    uint32_t rounds = 0;
};

}  // namespace

struct qtask_server_s {
    qtask_server_opts opts{};
    std::vector<SSession> sess;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<uint64_t, qtask_result> results;
    std::unordered_map<uint64_t, int32_t> pending_ticket;  // ticket -> session
    uint64_t next_ticket = 1;
    uint64_t used = 0;
    uint64_t peak_used = 0;
    int32_t resident = 0;
    std::vector<int32_t> waiting;        // planned requests waiting for memory, in start order
    std::vector<int32_t> replan;         // waiting requests whose session was evicted meanwhile
    bool stop = false;
    double t0 = 0;
    std::thread worker;
    hipStream_t bstream = nullptr;       // small-session batches
    hipEvent_t bdone = nullptr;
    bool tick_inflight = false;
    std::vector<int32_t> tick_sessions;
    BatchTables tables;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::atomic<uint64_t> n_batched{0}, n_streamed{0}, n_ticks{0};
    std::string error;

    double clock() const { return now_ms() - t0; }
    void run();
    int start_small_tick(std::vector<int32_t> &ready, std::vector<int32_t> &group);
    int launch_rounds(int dtype, bool mf, uint32_t threads, uint32_t lds, uint32_t rounds, uint32_t groups);
    void finish(int32_t sid, double done_ms);
    int admit(int32_t sid, uint64_t need);
    void evict(int32_t victim);
    int32_t lru_victim(int32_t except) const;
};

namespace {

int apply_edit(Session *s, const qtask_edit &e) {
    auto &c = s->circ;
    uint64_t lid = 0, out = 0;
    switch (e.op) {
    case 0: {
        int rc = c.level_at(e.level, &lid);
        if (rc) return rc;
        return c.insert_gate(lid, e.kind, e.qubits, e.nq, e.params, e.np, &out);
    }
    case 1: {
        int rc = c.level_at(e.level, &lid);
        if (rc) return rc;
        for (size_t i = 0; i < c.num_levels(); ++i) {
            const auto &lv = c.level_by_index(i);
            if (lv.id != lid) continue;
            if (e.gate_index >= lv.gates.size()) return QTASK_E_NOTFOUND;
            return c.remove_gate(lv.gates[e.gate_index]);
        }
        return QTASK_E_NOTFOUND;
    }
    case 2: {
        uint64_t after = QTASK_FRONT;
        if (e.level != UINT64_MAX) {
            int rc = c.level_at(e.level, &after);
            if (rc) return rc;
        }
        return c.insert_level(after, &out);
    }
    case 3: {
        int rc = c.level_at(e.level, &lid);
        if (rc) return rc;
        return c.remove_level(lid);
    }
    default:
        return QTASK_E_ARG;
    }
}

}  // namespace

// Least recently used resident session that is idle (nothing running,
// nothing planned, nothing queued), or -1.  Called with the lock held.
int32_t qtask_server_s::lru_victim(int32_t except) const {
    int32_t victim = -1;
    for (size_t i = 0; i < sess.size(); ++i) {
        const SSession &o = sess[i];
        if (int32_t(i) == except || !o.resident || o.busy || !o.q.empty()) continue;
        if (victim < 0 || o.last_used < sess[victim].last_used) victim = int32_t(i);
    }
    return victim;
}

// Free a resident session's device memory (its next update re-simulates
// from the start).  Called with the lock held; the session is not busy, or
// busy but neither running nor committed.
void qtask_server_s::evict(int32_t victim) {
    SSession &v = sess[victim];
    v.s->release_device();
    used -= v.bytes;
    v.bytes = 0;
    v.resident = false;
    --resident;
}

// Charge `need` bytes (the session's footprint after its planned update):
// 1 admitted (resident, charged at least `need`), 0 must wait for memory,
// -1 can never fit the budget.  Called with the lock held.
int qtask_server_s::admit(int32_t sid, uint64_t need) {
    SSession &ss = sess[sid];
    if (need > opts.budget_bytes) return -1;
    const uint64_t have = ss.resident ? ss.bytes : 0;
    if (need <= have) return 1;
    const uint64_t extra = need - have;
    while (used + extra > opts.budget_bytes) {
        const int32_t victim = lru_victim(sid);
        if (victim < 0) return 0;
        evict(victim);
    }
    if (!ss.resident) {
        ss.resident = true;
        ++resident;
    }
    ss.bytes = need;
    used += extra;
    peak_used = std::max(peak_used, used);
    return 1;
}

void qtask_server_s::finish(int32_t sid, double done_ms) {
    SSession &ss = sess[sid];
    Session *s = ss.s;
    qtask_result r{};
    r.ticket = ss.cur.ticket;
    r.session = sid;
    r.submit_ms = ss.cur.submit_ms;
    r.start_ms = ss.start_ms;
    r.status = ss.status;
    if (ss.status == QTASK_E_DEVICE) s->invalidate();
    if (ss.status == QTASK_OK) {
        s->finish_prepared_host();
        uint64_t h = 0;
        if (s->hash(&h) == QTASK_OK) r.state_hash = h;
    }
    r.done_ms = done_ms;
    r.latency_ms = done_ms - ss.cur.submit_ms;
    r.stats = s->last;
    r.stats.wall_ms = done_ms - ss.start_ms;
    const uint64_t nb = s->device_bytes();
    std::lock_guard<std::mutex> lk(mu);
    // charge what the session holds now: no more than admitted (the
    // admission charged its footprint after this update), less when the
    // update shrank it
    if (ss.resident) {
        used = used - ss.bytes + nb;
        ss.bytes = nb;
        peak_used = std::max(peak_used, used);
        while (used > opts.budget_bytes) {
            const int32_t victim = lru_victim(sid);
            if (victim < 0) break;
            evict(victim);
        }
    }
    ss.busy = false;
    ss.waiting = false;
    ss.last_used = done_ms;
    results[r.ticket] = r;
    pending_ticket.erase(r.ticket);
    cv_done.notify_all();
}

int qtask_server_s::launch_rounds(int dtype, bool mf, uint32_t threads, uint32_t lds, uint32_t rounds,
                                  uint32_t groups) {
    // rounds and groups are capacities: the tables say how much work each round has
    const GraphKey key{dtype, int(mf), int(threads), int(rounds), int(groups)};
    auto enqueue = [&]() -> int {
        for (uint32_t r = 0; r < rounds; ++r) {
            if (qtask::launch_pass_batch(dtype, mf, tables.d_items + size_t(r) * kMaxItems, tables.d_counts + r, groups,
                                         threads, lds, bstream) != hipSuccess)
                return QTASK_E_DEVICE;
            if (qtask::launch_batch_sums(tables.d_sums + size_t(r) * kMaxItems, tables.d_counts + tables.rounds + r,
                                         kMaxItems, bstream) != hipSuccess)
                return QTASK_E_DEVICE;
        }
        return QTASK_OK;
    };
    if (!opts.use_graph) return enqueue();
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hipStreamBeginCapture(bstream, hipStreamCaptureModeThreadLocal) != hipSuccess) return QTASK_E_DEVICE;
        int rc = enqueue();
        const hipError_t e = hipStreamEndCapture(bstream, &g);
        if (rc != QTASK_OK || e != hipSuccess) return QTASK_E_DEVICE;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return QTASK_E_DEVICE;
        }
        (void)hipGraphDestroy(g);
        it = graphs.emplace(key, ge).first;
    }
    return hipGraphLaunch(it->second, bstream) == hipSuccess ? QTASK_OK : QTASK_E_DEVICE;
}

// Build the round tables for the ready small sessions (all prepared) and
// launch them; returns after enqueueing.
int qtask_server_s::start_small_tick(std::vector<int32_t> &ready, std::vector<int32_t> &group) {
    group.clear();
    if (ready.empty()) return QTASK_OK;
    // one tile shape per tick: the shape of the oldest ready session
    auto shape = [&](int32_t sid) {
        const Session *s = sess[sid].s;
        return s->launches.empty() ? -1 : s->launches[0].b;
    };
    const int dtype = sess[ready[0]].s->dtype;
    int b = -1;
    for (int32_t sid : ready)
        if (sess[sid].s->dtype == dtype && shape(sid) >= 0) { b = shape(sid); break; }
    std::vector<int32_t> rest;
    for (int32_t sid : ready) {
        const int bs = shape(sid);
        if (sess[sid].s->dtype == dtype && (bs == b || bs < 0) && group.size() < kMaxItems) group.push_back(sid);
        else rest.push_back(sid);
    }
    ready.swap(rest);
    if (b < 0) b = QK_MIN_TILE_BITS;  // no pass work in this tick
    const uint32_t threads = 1u << (b - QK_G);
    // the matrix-core kernel variant when any pass of the tick needs it (it
    // runs the other passes in the vector-ALU body, as their own launch would)
    bool mf = false;
    for (int32_t sid : group)
        for (const auto &l : sess[sid].s->launches) mf = mf || (l.n_tiles > 0 && qtask::pass_uses_mf(dtype, l.args));
    const uint32_t lds = qtask::pass_lds_bytes(dtype, mf, b);
    size_t max_rounds = 0;
    uint32_t max_groups = 1;
    for (int32_t sid : group) {
        const auto &ls = sess[sid].s->launches;
        max_rounds = std::max(max_rounds, ls.size());
        for (const auto &l : ls) max_groups = std::max(max_groups, l.n_tiles);
    }
    uint32_t rcap = kRoundCaps[2];
    for (uint32_t c : kRoundCaps)
        if (c >= max_rounds) { rcap = c; break; }
    // the tables are sized for the largest round capacity
    const uint32_t tr = kRoundCaps[2];
    if (!tables.d_items) {
        if (hipMalloc(&tables.d_items, sizeof(KBatchItem) * kMaxItems * tr) != hipSuccess ||
            hipMalloc(&tables.d_sums, sizeof(KSumItem) * kMaxItems * tr) != hipSuccess ||
            hipMalloc(&tables.d_counts, sizeof(uint32_t) * 2 * tr) != hipSuccess ||
            hipHostMalloc(&tables.h_items, sizeof(KBatchItem) * kMaxItems * tr) != hipSuccess ||
            hipHostMalloc(&tables.h_sums, sizeof(KSumItem) * kMaxItems * tr) != hipSuccess ||
            hipHostMalloc(&tables.h_counts, sizeof(uint32_t) * 2 * tr) != hipSuccess)
            return QTASK_E_NOMEM;
        tables.rounds = tr;
    }
    // the per-round workgroup total can exceed one session's tiles
    for (size_t r0 = 0; r0 < max_rounds; r0 += rcap) {
        uint32_t need_groups = 1;
        std::memset(tables.h_counts, 0, sizeof(uint32_t) * 2 * tr);
        for (uint32_t r = 0; r < rcap; ++r) {
            uint32_t ni = 0, ns = 0, tiles = 0;
            for (int32_t sid : group) {
                Session *s = sess[sid].s;
                const size_t li = r0 + r;
                if (li >= s->launches.size()) continue;
                const Session::Launch &l = s->launches[li];
                if (l.n_tiles > 0) {
                    KBatchItem &it = tables.h_items[size_t(r) * kMaxItems + ni++];
                    it.args = l.args;
                    it.tile_begin = tiles;
                    it.n_tiles = l.n_tiles;
                    it.threads = threads;
                    it.pad = 0;
                    tiles += l.n_tiles;
                }
                if (l.after == 1) {
                    KSumItem &si = tables.h_sums[size_t(r) * kMaxItems + ns++];
                    double *norm = nullptr, *scale = nullptr;
                    s->sum_targets(l, &si.partials, &norm, &scale);
                    si.norm_out = norm;
                    si.scale_out = scale;
                    si.n = l.n_tiles;
                    si.pad = 0;
                }
            }
            tables.h_counts[r] = ni;
            tables.h_counts[tr + r] = ns;
            need_groups = std::max(need_groups, tiles);
        }
        uint32_t gcap = 0;
        for (uint32_t c : kGroupCaps)
            if (c >= need_groups) { gcap = c; break; }
        if (gcap == 0) return QTASK_E_UNSUPPORTED;
        if (hipMemcpyAsync(tables.d_items, tables.h_items, sizeof(KBatchItem) * kMaxItems * rcap,
                           hipMemcpyHostToDevice, bstream) != hipSuccess ||
            hipMemcpyAsync(tables.d_sums, tables.h_sums, sizeof(KSumItem) * kMaxItems * rcap, hipMemcpyHostToDevice,
                           bstream) != hipSuccess ||
            hipMemcpyAsync(tables.d_counts, tables.h_counts, sizeof(uint32_t) * 2 * tr, hipMemcpyHostToDevice,
                           bstream) != hipSuccess)
            return QTASK_E_DEVICE;
        int rc = launch_rounds(dtype, mf, threads, lds, rcap, gcap);
        if (rc != QTASK_OK) return rc;
        // the staging buffers are reused by the next chunk: wait for the copies
        if (r0 + rcap < max_rounds && hipStreamSynchronize(bstream) != hipSuccess) return QTASK_E_DEVICE;
    }
    for (int32_t sid : group) {
        Session *s = sess[sid].s;
        if (s->needs_final() && s->enqueue_final(bstream) != QTASK_OK) return QTASK_E_DEVICE;
    }
    if (hipEventRecord(bdone, bstream) != hipSuccess) return QTASK_E_DEVICE;
    tick_sessions = group;
    tick_inflight = true;
    n_ticks += 1;
    n_batched += group.size();
    return QTASK_OK;
}

void qtask_server_s::run() {
    (void)hipSetDevice(opts.device);
    int inflight_large = 0;
    std::vector<int32_t> small_ready;
    while (true) {
        // 1. take new work: oldest request first, as far as memory and launch
        //    slots allow
        std::vector<int32_t> starts;
        {
            std::unique_lock<std::mutex> lk(mu);
            const bool any_busy = tick_inflight || inflight_large > 0 || !waiting.empty() || !replan.empty();
            if (!any_busy && small_ready.empty()) {
                cv_work.wait(lk, [&] {
                    if (stop) return true;
                    for (const auto &ss : sess)
                        if (!ss.busy && !ss.q.empty()) return true;
                    return false;
                });
            }
            if (stop && !any_busy && small_ready.empty()) {
                bool pending = false;
                for (const auto &ss : sess) pending = pending || !ss.q.empty();
                if (!pending) return;
            }
            std::vector<int32_t> order;
            for (size_t i = 0; i < sess.size(); ++i)
                if (!sess[i].busy && !sess[i].q.empty()) order.push_back(int32_t(i));
            // oldest first, or expected-shortest first with the estimate
            // discounted by waiting time (only the worker touches a session's
            // circuit, so reading its size here is safe)
            const double now = clock();
            auto key = [&](int32_t sid) {
                const SSession &ss = sess[sid];
                const double submit = ss.q.front().submit_ms;
                if (opts.order == 0) return submit;
                const double cost = std::ldexp(double(std::max<size_t>(1, ss.s->circ.num_levels())), ss.s->n_int);
                return cost / (1.0 + std::max(0.0, now - submit) / kAgingMs);
            };
            std::vector<std::pair<double, double>> keys(sess.size());
            for (int32_t sid : order) keys[size_t(sid)] = {key(sid), sess[sid].q.front().submit_ms};
            std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return keys[size_t(a)] < keys[size_t(b)]; });
            for (int32_t sid : order) {
                SSession &ss = sess[sid];
                if (!ss.small && inflight_large >= opts.max_inflight) continue;
                ss.busy = true;
                ss.batched = false;
                ss.waiting = true;
                ss.cur = std::move(ss.q.front());
                ss.q.pop_front();
                ss.counted = !ss.small;
                if (ss.counted) ++inflight_large;
                starts.push_back(sid);
            }
        }
        auto fail = [&](int32_t sid, int code, bool rollback) {
            SSession &ss = sess[sid];
            if (rollback) ss.s->rollback_edit_point();
            ss.status = code;
            if (ss.counted) --inflight_large;
            ss.counted = false;
            finish(sid, clock());
        };
        // waiting sessions whose memory was freed while they waited lost
        // their plans: plan them again (now a full simulation)
        for (int32_t sid : replan) {
            SSession &ss = sess[sid];
            const int rc = ss.s->plan_update(false);
            if (rc != QTASK_OK) {
                fail(sid, rc, true);
                continue;
            }
            waiting.push_back(sid);
        }
        replan.clear();
        // 2. apply the edits and plan the update on the host (outside the
        //    lock: only the worker touches a busy session).  A request is
        //    all or nothing: a failed edit or plan undoes its edits.
        for (int32_t sid : starts) {
            SSession &ss = sess[sid];
            ss.start_ms = clock();
            ss.status = QTASK_OK;
            ss.s->save_edit_point();
            int rc = QTASK_OK;
            for (size_t i = 0; i < ss.cur.edits.size() && rc == QTASK_OK; ++i) rc = apply_edit(ss.s, ss.cur.edits[i]);
            if (rc == QTASK_OK) rc = ss.s->init_device();
            if (rc == QTASK_OK) rc = ss.s->ensure_tuned();
            if (rc == QTASK_OK) rc = ss.s->plan_update(false);
            if (rc != QTASK_OK) {
                if (rc == QTASK_E_DEVICE) ss.s->invalidate();
                fail(sid, rc, true);
                continue;
            }
            ss.waiting = true;
            waiting.push_back(sid);
        }
        // 3. admission of the planned requests, oldest start first, by the
        //    bytes each session holds after its update
        std::vector<int32_t> commits, never;
        {
            std::lock_guard<std::mutex> lk(mu);
            std::vector<int32_t> still;
            for (int32_t sid : waiting) {
                const int adm = admit(sid, sess[sid].s->bytes_after_commit());
                if (adm > 0) commits.push_back(sid);
                else if (adm < 0) never.push_back(sid);
                else still.push_back(sid);
            }
            // Nothing running can free memory and nothing was admitted: the
            // waiting sessions block one another.  Free the others' memory
            // (they re-simulate later) so that the oldest one fits.
            if (commits.empty() && !still.empty() && !tick_inflight && small_ready.empty()) {
                bool running = false;
                for (const auto &o : sess) running = running || (o.busy && !o.waiting);
                if (!running) {
                    std::vector<int32_t> keep{still[0]};
                    for (size_t i = 1; i < still.size(); ++i) {
                        if (sess[still[i]].resident) {
                            evict(still[i]);
                            replan.push_back(still[i]);
                        } else {
                            keep.push_back(still[i]);
                        }
                    }
                    still.swap(keep);
                    if (admit(still[0], sess[still[0]].s->bytes_after_commit()) > 0) {
                        commits.push_back(still[0]);
                        still.erase(still.begin());
                    }
                }
            }
            waiting.swap(still);
        }
        for (int32_t sid : never) fail(sid, QTASK_E_NOMEM, true);
        // 4. commit (allocate, upload) and launch
        for (int32_t sid : commits) {
            SSession &ss = sess[sid];
            ss.waiting = false;
            int rc = ss.s->commit_device();
            if (rc != QTASK_OK) {
                if (rc == QTASK_E_DEVICE) ss.s->invalidate();
                fail(sid, rc, rc != QTASK_E_DEVICE);
                continue;
            }
            // the batched kernel runs pass launches of every kernel variant;
            // plans with block copies (sparse checkpoints) run on the
            // session's own stream
            bool own = ss.s->opts.ckpt_delta != 0;
            for (const auto &l : ss.s->launches) own = own || l.kind != 0;
            ss.batched = ss.small && !own;
            if (ss.batched) {
                // plan uploads went to the session's stream
                if (hipStreamSynchronize(ss.s->stream) != hipSuccess) {
                    ss.s->invalidate();
                    fail(sid, QTASK_E_DEVICE, false);
                    continue;
                }
                small_ready.push_back(sid);
            } else if (ss.s->enqueue_prepared(ss.s->stream) != QTASK_OK ||
                       hipEventRecord(ss.done, ss.s->stream) != hipSuccess) {
                (void)hipStreamSynchronize(ss.s->stream);
                ss.s->invalidate();
                fail(sid, QTASK_E_DEVICE, false);
            } else {
                n_streamed += 1;
            }
        }
        // 3. a batched tick when none is running; sessions that become ready
        //    meanwhile join the next one
        if (!tick_inflight && !small_ready.empty()) {
            std::vector<int32_t> group;
            const int rc = start_small_tick(small_ready, group);
            if (rc != QTASK_OK) {
                (void)hipStreamSynchronize(bstream);
                for (int32_t sid : group) {
                    sess[sid].status = rc;
                    finish(sid, clock());
                }
                tick_inflight = false;
            }
        }
        // 4. completions
        bool progressed = false;
        for (size_t i = 0; i < sess.size(); ++i) {
            SSession &ss = sess[i];
            // only launched requests on the session's own stream: batched
            // ones finish with their tick, planned ones still wait for memory
            if (!ss.busy || ss.batched || ss.waiting) continue;
            const hipError_t q = hipEventQuery(ss.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) ss.status = QTASK_E_DEVICE;
            if (ss.counted) --inflight_large;
            ss.counted = false;
            finish(int32_t(i), clock());
            progressed = true;
        }
        if (tick_inflight) {
            const hipError_t q = hipEventQuery(bdone);
            if (q != hipErrorNotReady) {
                const double t = clock();
                for (int32_t sid : tick_sessions) {
                    if (q != hipSuccess) sess[sid].status = QTASK_E_DEVICE;
                    finish(sid, t);
                }
                tick_sessions.clear();
                tick_inflight = false;
                progressed = true;
            }
        }
        if (!progressed && starts.empty() && (tick_inflight || inflight_large > 0))
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

extern "C" {

int qtask_server_opts_default(qtask_server_opts *o) {
    if (!o) return QTASK_E_ARG;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(*o);
    o->device = 0;
    o->budget_bytes = uint64_t(256) << 30;
    o->max_inflight = 4;
    o->small_qubits = 16;
    o->use_graph = 1;
    return QTASK_OK;
}

int qtask_server_create(const qtask_server_opts *user, qtask_server_t *out) {
    if (!out) return QTASK_E_ARG;
    qtask_server_opts o;
    qtask_server_opts_default(&o);
    if (user) {
        if (user->struct_size != sizeof(qtask_server_opts)) return QTASK_E_ARG;
        o = *user;
    }
    if (o.max_inflight < 1 || o.small_qubits < 0 || o.device < 0 || o.order < 0 || o.order > 1) return QTASK_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || o.device >= count) {
        (void)hipGetLastError();
        return QTASK_E_DEVICE;
    }
    auto *s = new qtask_server_s();
    s->opts = o;
    s->t0 = now_ms();
    if (hipSetDevice(o.device) != hipSuccess || hipStreamCreateWithFlags(&s->bstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->bdone, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return QTASK_E_DEVICE;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return QTASK_OK;
}

int qtask_server_destroy(qtask_server_t s) {
    if (!s) return QTASK_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->opts.device);
    (void)hipStreamSynchronize(s->bstream);
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &ss : s->sess) {
        if (ss.done) (void)hipEventDestroy(ss.done);
        qtask::set_server_owned(ss.handle, false);
        qtask_destroy(ss.handle);
    }
    if (s->tables.d_items) {
        (void)hipFree(s->tables.d_items);
        (void)hipFree(s->tables.d_sums);
        (void)hipFree(s->tables.d_counts);
        (void)hipHostFree(s->tables.h_items);
        (void)hipHostFree(s->tables.h_sums);
        (void)hipHostFree(s->tables.h_counts);
    }
    (void)hipEventDestroy(s->bdone);
    (void)hipStreamDestroy(s->bstream);
    delete s;
    return QTASK_OK;
}

int qtask_server_open(qtask_server_t sv, int n_qubits, qtask_dtype dtype, const qtask_opts *user, uint64_t n_levels,
                      uint64_t n_gates, const int32_t *kinds, const int32_t *qubits, const int32_t *nq,
                      const double *params, const uint64_t *level_of_gate, int32_t *session_out) {
    if (!sv || !session_out) return QTASK_E_ARG;
    if (n_gates > 0 && (!kinds || !qubits || !nq || !params || !level_of_gate)) return QTASK_E_ARG;
    qtask_opts o;
    qtask_opts_default(&o);
    if (user) o = *user;
    o.device = sv->opts.device;
    o.stream = nullptr;
    qtask_t h = nullptr;
    int rc = qtask_create(n_qubits, dtype, &o, &h);
    if (rc != QTASK_OK) return rc;
    // the server owns the session from here on: through the handle that
    // qtask_server_session lends, the caller can only query it
    Session *s = qtask::session_of(h);
    qtask::set_server_owned(h, true);
    auto drop = [&](int code) {
        qtask::set_server_owned(h, false);
        qtask_destroy(h);
        return code;
    };
    std::vector<uint64_t> levels(n_levels);
    uint64_t prev = QTASK_FRONT;
    for (uint64_t i = 0; i < n_levels; ++i) {
        rc = s->circ.insert_level(prev, &levels[i]);
        if (rc != QTASK_OK) return drop(rc);
        prev = levels[i];
    }
    for (uint64_t g = 0; g < n_gates; ++g) {
        if (level_of_gate[g] >= n_levels) return drop(QTASK_E_ARG);
        const int np = qtask::kind_nparams(kinds[g]);
        uint64_t gid = 0;
        rc = s->circ.insert_gate(levels[level_of_gate[g]], kinds[g], qubits + 3 * g, nq[g], params + 3 * g,
                                 np < 0 ? 0 : np, &gid);
        if (rc != QTASK_OK) return drop(rc);
    }
    SSession ss;
    ss.s = s;
    ss.handle = h;
    ss.small = n_qubits < sv->opts.small_qubits;
    (void)hipSetDevice(sv->opts.device);
    if (hipEventCreateWithFlags(&ss.done, hipEventDisableTiming) != hipSuccess) return drop(QTASK_E_DEVICE);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->sess.push_back(ss);
    *session_out = int32_t(sv->sess.size() - 1);
    return QTASK_OK;
}

int qtask_server_submit(qtask_server_t sv, int32_t session, const qtask_edit *edits, int n_edits,
                        uint64_t *ticket_out) {
    if (!sv || !ticket_out || n_edits < 0 || (n_edits > 0 && !edits)) return QTASK_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (session < 0 || size_t(session) >= sv->sess.size()) return QTASK_E_NOTFOUND;
    Request r;
    r.ticket = sv->next_ticket++;
    r.sid = session;
    r.edits.assign(edits, edits + n_edits);
    r.submit_ms = sv->clock();
    sv->pending_ticket[r.ticket] = session;
    *ticket_out = r.ticket;
    sv->sess[session].q.push_back(std::move(r));
    sv->cv_work.notify_all();
    return QTASK_OK;
}

int qtask_server_wait(qtask_server_t sv, uint64_t ticket, double timeout_ms, qtask_result *out) {
    if (!sv || !out) return QTASK_E_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return sv->results.count(ticket) > 0; };
    if (!ready() && !sv->pending_ticket.count(ticket)) return QTASK_E_NOTFOUND;
    if (timeout_ms < 0) sv->cv_done.wait(lk, ready);
    else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return QTASK_E_BUSY;
    *out = sv->results.at(ticket);
    return QTASK_OK;
}

int qtask_server_poll(qtask_server_t sv, uint64_t ticket, int *done, qtask_result *out) {
    if (!sv || !done || !out) return QTASK_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) {
        if (!sv->pending_ticket.count(ticket)) return QTASK_E_NOTFOUND;
        *done = 0;
        return QTASK_OK;
    }
    *done = 1;
    *out = it->second;
    return QTASK_OK;
}

int qtask_server_drain(qtask_server_t sv) {
    if (!sv) return QTASK_E_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->pending_ticket.empty(); });
    return QTASK_OK;
}

int qtask_server_session(qtask_server_t sv, int32_t session, qtask_t *out) {
    if (!sv || !out) return QTASK_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (session < 0 || size_t(session) >= sv->sess.size()) return QTASK_E_NOTFOUND;
    const SSession &ss = sv->sess[session];
    if (ss.busy || !ss.q.empty()) return QTASK_E_BUSY;
    *out = ss.handle;
    return QTASK_OK;
}

int qtask_server_usage(qtask_server_t sv, uint64_t *bytes, int32_t *resident) {
    if (!sv || !bytes || !resident) return QTASK_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *bytes = sv->used;
    *resident = sv->resident;
    return QTASK_OK;
}

int qtask_server_paths(qtask_server_t sv, uint64_t *batched, uint64_t *streamed, uint64_t *ticks) {
    if (!sv || !batched || !streamed || !ticks) return QTASK_E_ARG;
    *batched = sv->n_batched.load();
    *streamed = sv->n_streamed.load();
    *ticks = sv->n_ticks.load();
    return QTASK_OK;
}

int qtask_server_peak_bytes(qtask_server_t sv, uint64_t *peak) {
    if (!sv || !peak) return QTASK_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *peak = sv->peak_used;
    return QTASK_OK;
}

}  // extern "C"
