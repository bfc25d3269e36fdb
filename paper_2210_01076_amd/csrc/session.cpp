// Session: full and incremental state update on one device.
//
// The circuit is cut into segments of K levels.  Each segment has its own
// plan (a pure function of the segment's gates), and the state after each
// segment boundary can be kept on the device as a checkpoint (the paper keeps
// per-net state vectors for the same purpose, Section III-F).  An update
// after circuit modifiers restores the newest valid checkpoint at or before
// the first modified level and re-runs the segments from there; when the set
// of blocks the modifiers can reach is closed under every replayed gate, only
// the tiles holding those blocks are re-run and only those blocks are stored
// (the paper's frontier-and-reachability update, Section III-E).  Because
// plans, kernels and the tile arithmetic do not depend on which tiles run,
// the incremental result is bitwise identical to a full re-simulation.
#include "session.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <future>
#include <sstream>

#include "device.h"

namespace qtask {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

#define HIPCHK(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            last_error = std::string(#expr) + ": " + hipGetErrorString(e_); \
            return QTASK_E_DEVICE;                                          \
        }                                                                   \
    } while (0)

Session::Session(int n_, int dtype_, const qtask_opts &o)
    : circ(n_), n(n_), n_int(std::max(n_, QK_MIN_TILE_BITS)), dtype(dtype_), elem(dtype_ == QTASK_C128 ? 16 : 8),
      opts(o), plan_only(o.device == QTASK_DEVICE_NONE) {
    last.struct_size = sizeof(qtask_stats);
}

Session::~Session() {
    if (plan_only) return;
    (void)hipSetDevice(opts.device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto &kv : plan_cache_) dfree(kv.second.dev);
    dfree(state_.p);
    for (auto &kv : ckpts_) dfree(kv.second.buf.p);
    dfree(d_partials_);
    dfree(d_scalars_);
    dfree(d_u64_);
    dfree(d_mask_);
    dfree(d_tiles_);
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void *Session::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (opts.alloc) {
        // the kernels read plan records and operands with aligned vector loads
        void *p = opts.alloc(bytes, opts.alloc_ctx);
        if (p && (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
            if (opts.free) opts.free(p, opts.alloc_ctx);
            last_error = "alloc hook returned memory not aligned to 256 bytes";
            return nullptr;
        }
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Session::dfree(void *p) {
    if (!p) return;
    if (opts.free) opts.free(p, opts.alloc_ctx);
    else (void)hipFree(p);
}

int Session::init_device() {
    if (plan_only || dev_ready_) return QTASK_OK;
    HIPCHK(hipSetDevice(opts.device));
    if (opts.stream) {
        stream = static_cast<hipStream_t>(opts.stream);
    } else {
        HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        own_stream = true;
    }
    HIPCHK(hipEventCreate(&ev0_));
    HIPCHK(hipEventCreate(&ev1_));
    dev_ready_ = true;
    return QTASK_OK;
}

// With at most max_ckpts checkpoints, every stride-th boundary keeps one.
// The stride only grows (when the boundaries outgrow it), so a circuit that
// gains or loses a segment keeps its stored boundaries and their checkpoints.
bool Session::stores_ckpt(size_t j, size_t S) const {
    if (j == 0 || j >= S) return false;
    if (opts.max_ckpts < 0) return true;
    if (opts.max_ckpts == 0) return false;
    const size_t nb = S - 1;
    size_t stride = std::max<size_t>(ckpt_stride_, 1);
    while (nb / stride > size_t(opts.max_ckpts)) ++stride;
    ckpt_stride_ = stride;
    return j % stride == 0;
}

uint64_t Session::planned_bytes() const {
    const size_t S = num_segments();
    uint64_t b = state_bytes();
    for (size_t j = 1; j < S; ++j)
        if (stores_ckpt(j, S)) b += state_bytes();
    return b + (uint64_t(1) << 20);
}

uint64_t Session::device_bytes() const {
    uint64_t b = state_.bytes;
    for (const auto &kv : ckpts_) b += kv.second.buf.bytes + kv.second.d_blocks.bytes;
    b += restore_cap_ * sizeof(uint32_t);
    for (const auto &kv : plan_cache_) b += kv.second.dev_bytes;
    b += (scalars_cap_ + partials_cap_) * sizeof(double) + u64_cap_ * sizeof(unsigned long long) +
         tiles_cap_ * sizeof(uint32_t) + mask_cap_ * sizeof(uint64_t);
    return b;
}

std::vector<LGate> Session::level_ops(size_t lo, size_t hi) const {
    std::vector<LGate> ops;
    for (size_t li = lo; li < hi; ++li) {
        const Level &lv = circ.level_by_index(li);
        std::vector<const Gate *> gs;
        for (uint64_t gid : lv.gates) gs.push_back(&circ.gate(gid));
        // canonical order inside a level: by lowest qubit (the gates of a
        // level act on disjoint qubits, so this is a total order)
        std::sort(gs.begin(), gs.end(), [](const Gate *a, const Gate *b) {
            const int la = *std::min_element(a->q, a->q + a->nq);
            const int lb = *std::min_element(b->q, b->q + b->nq);
            return la < lb;
        });
        for (const Gate *g : gs) {
            auto it = lowered_.find(g->id);
            if (it == lowered_.end()) it = lowered_.emplace(g->id, lower_gate(g->kind, g->q, g->p, g->id)).first;
            ops.push_back(it->second);
        }
    }
    if (lowered_.size() > 2 * circ.num_gates() + 1024) {
        for (auto it = lowered_.begin(); it != lowered_.end();)
            it = circ.has_gate(it->first) ? std::next(it) : lowered_.erase(it);
    }
    return ops;
}

// Cut the circuit at its anchor levels.  The first time (no anchors) every
// K-th level becomes an anchor; levels appended after the last anchor are cut
// every K levels; a segment that grew to 2K levels through insertions is split.
// The cut is a function of the circuit and the anchor set alone, and running
// it again on what it returns changes nothing: an anchor on the last level
// (which ends no segment) stays an anchor, since dropping it would move the
// start of the tail and so the cuts of a second run.  An incremental update
// and the full re-simulation that follows it then run the same segments.
void Session::build_segments(const PlanParams &pp) {
    segs_.clear();
    const size_t D = circ.num_levels();
    const size_t Kz = size_t(K());
    size_t last_anchor = SIZE_MAX;
    for (size_t i = 0; i < D; ++i)
        if (anchors_.count(circ.level_by_index(i).id)) last_anchor = i;
    std::unordered_set<uint64_t> used;
    size_t lo = 0;
    for (size_t i = 0; i < D; ++i) {
        const uint64_t id = circ.level_by_index(i).id;
        const size_t len = i - lo + 1;
        const bool tail = last_anchor == SIZE_MAX || i > last_anchor;
        const bool cut = anchors_.count(id) || len >= 2 * Kz || (tail && len >= Kz);
        if (cut && i + 1 < D) {
            Seg sg;
            sg.lo = lo;
            sg.hi = i + 1;
            sg.anchor = id;
            segs_.push_back(sg);
            used.insert(id);
            lo = i + 1;
        } else if (anchors_.count(id)) {
            used.insert(id);  // the last level
        }
    }
    if (D > 0) {
        Seg sg;
        sg.lo = lo;
        sg.hi = D;
        sg.anchor = 0;
        segs_.push_back(sg);
    }
    anchors_ = used;
    for (auto &sg : segs_) {
        uint64_t k = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { k = hash_mix(k, v); };
        mix(uint64_t(pp.b) | uint64_t(pp.c) << 8 | uint64_t(pp.fusion) << 16 | uint64_t(pp.fuse_k) << 24 |
            uint64_t(pp.dtype) << 32 | uint64_t(pp.relabel) << 40);
        for (size_t i = sg.lo; i < sg.hi; ++i) {
            const Level &lv = circ.level_by_index(i);
            mix(lv.id);
            mix(lv.version);
        }
        sg.key = k;
    }
}

size_t Session::slot_of(uint64_t anchor) {
    if (anchor == 0) return 0;
    auto it = slots_.find(anchor);
    if (it != slots_.end()) return it->second;
    const size_t sl = next_slot_++;
    slots_.emplace(anchor, sl);
    return sl;
}

// Blocks of 2^block_bits amplitudes that a segment's plan can change, by
// the kernel form of its ops (empty: every block).  A fused dense stage, a
// store permutation, a segment scalar and a renormalised complex64 segment
// change every block; otherwise each op changes the blocks it rewrites.
const std::vector<uint32_t> &Session::written_blocks(const SegmentPlan &sp) {
    auto it = wsets_.find(sp.hash);
    if (it != wsets_.end()) return it->second;
    std::vector<uint32_t> out;
    const int beta = std::min(opts.block_bits, n_int);
    const uint64_t nblocks = uint64_t(1) << (n_int - beta);
    bool all = dtype == QTASK_C64 && opts.renorm != 0;
    BlockSet w(nblocks);
    for (const auto &p : sp.passes) {
        if (all) break;
        if (p.relabels()) { all = true; break; }
        for (const auto &st : p.stages) {
            if (!st.U.empty() || st.mfma) { all = true; break; }
            for (const auto &g : st.ops) {
                if (rewrites_every_block(g, beta)) {
                    all = true;
                    break;
                }
                for_rewritten_blocks(g, beta, nblocks, [&](uint64_t k) { w.set(k); });
            }
            if (all) break;
        }
    }
    if (!all && w.count() < nblocks) out = w.list();
    uint64_t key = 0;
    if (!out.empty()) {
        key = 0x44454c5441ull;
        for (uint32_t b : out) key = hash_mix(key, b);
    }
    wkeys_[sp.hash] = key;
    return wsets_.emplace(sp.hash, std::move(out)).first->second;
}

// The checkpoint layout of boundary j (the state before segment j).
Session::CkptLayout Session::layout_of(size_t j) const {
    CkptLayout L;
    L.bytes = state_bytes();
    if (!opts.ckpt_delta) return L;
    // the blocks the segments since the previous stored boundary can change
    const size_t S = segs_.size();
    size_t i = j - 1;
    while (i >= 1 && !stores_ckpt(i, S)) --i;
    uint64_t ukey = 0x554e494f4eull;
    for (size_t s = i; s < j; ++s) {
        auto it = wsets_.find(plans_[s]->hash);
        if (it == wsets_.end() || it->second.empty()) return L;  // a segment that changes every block
        ukey = hash_mix(ukey, wkeys_.at(plans_[s]->hash));
    }
    const std::vector<uint32_t> *blocks = nullptr;
    if (j - i == 1) {
        blocks = &wsets_.at(plans_[i]->hash);
    } else {
        auto u = unions_.find(ukey);
        if (u == unions_.end()) {
            const int beta = std::min(opts.block_bits, n_int);
            BlockSet w(uint64_t(1) << (n_int - beta));
            for (size_t s = i; s < j; ++s)
                for (uint32_t b : wsets_.at(plans_[s]->hash)) w.set(b);
            u = unions_.emplace(ukey, w.list()).first;
        }
        blocks = &u->second;
        if (blocks->size() == (size_t(1) << (n_int - std::min(opts.block_bits, n_int)))) return L;
    }
    uint64_t key = 0x44454c5441ull;
    for (uint32_t b : *blocks) key = hash_mix(key, b);
    const int beta = std::min(opts.block_bits, n_int);
    L.full = false;
    L.blocks = blocks;
    L.wkey = key;
    L.bytes = uint64_t(blocks->size()) * (uint64_t(1) << beta) * elem;
    return L;
}

int Session::ensure_state() {
    if (state_.p) return QTASK_OK;
    state_.p = dalloc(state_bytes());
    if (!state_.p) return QTASK_E_NOMEM;
    state_.bytes = state_bytes();
    return QTASK_OK;
}

int Session::upload_plan(SegmentPlan &sp) {
    if (plan_only) return QTASK_OK;
    sp.dev = dalloc(sp.blob.size());
    if (!sp.dev) return QTASK_E_NOMEM;
    sp.dev_bytes = sp.blob.size();
    HIPCHK(hipMemcpyAsync(sp.dev, sp.blob.data(), sp.blob.size(), hipMemcpyHostToDevice, stream));
    return QTASK_OK;
}

namespace {

bool same_gate(const LGate &a, const LGate &b) {
    if (a.kop != b.kop || a.nq != b.nq) return false;
    for (int j = 0; j < a.nq; ++j)
        if (a.q[j] != b.q[j]) return false;
    return a.m.size() == b.m.size() && std::memcmp(a.m.data(), b.m.data(), a.m.size() * sizeof(cd)) == 0;
}

bool same_pass(const PPass &a, const PPass &b) {
    if (a.qlist != b.qlist || a.stages.size() != b.stages.size()) return false;
    for (size_t p = 0; p < a.qlist.size(); ++p)
        if (a.out_pos(int(p)) != b.out_pos(int(p))) return false;
    for (size_t i = 0; i < a.stages.size(); ++i) {
        const PStage &x = a.stages[i], &y = b.stages[i];
        if (x.tbits != y.tbits || x.mfma != y.mfma || x.ops.size() != y.ops.size()) return false;
        if (x.U.size() != y.U.size() ||
            (!x.U.empty() && std::memcmp(x.U.data(), y.U.data(), x.U.size() * sizeof(cd)) != 0))
            return false;
        for (size_t k = 0; k < x.ops.size(); ++k)
            if (!same_gate(x.ops[k], y.ops[k])) return false;
    }
    return true;
}

// The store permutation of a relabelling pass as a sequence of exact
// exchanges of two positions (SWAP ops, in order): the amplitude at a
// position moves where the pass stores it.
std::vector<LGate> relabel_swaps(const PPass &p) {
    std::vector<LGate> out;
    if (!p.relabels()) return out;
    // cur[k] = position that now holds what was loaded from qlist[k]
    std::vector<int> cur(p.qlist);
    for (size_t k = 0; k < cur.size(); ++k) {
        const int want = p.out_pos(int(k));
        if (cur[k] == want) continue;
        // whichever tile bit sits at `want` trades places with bit k
        size_t j = 0;
        while (cur[j] != want) ++j;
        const int qa = cur[k], qb = want;
        out.push_back(lower_gate(QTASK_SWAP, std::array<int, 2>{qa, qb}.data(), nullptr, 0));
        std::swap(cur[k], cur[j]);
    }
    return out;
}

// f(BlockAction) for every op of the pass in program order; a fused dense
// stage is one op on all of its qubits; a relabelling pass ends with its
// store permutation
template <typename F>
void for_pass_actions(const PPass &p, int beta, F &&f) {
    for (const auto &st : p.stages) {
        if (!st.U.empty()) {
            std::vector<int> qs;
            for (int tb : st.tbits) qs.push_back(p.qlist[tb]);
            f(dense_action(qs, beta));
            continue;
        }
        for (const auto &g : st.ops) f(block_action(g, beta));
    }
    for (const auto &g : relabel_swaps(p)) f(block_action(g, beta));
}

uint64_t pext_tile(uint64_t x, const uint8_t *pos, uint32_t npos) {
    uint64_t t = 0;
    for (uint32_t k = 0; k < npos; ++k) t |= ((x >> pos[k]) & 1) << k;
    return t;
}

}  // namespace

// Decide whether the replay can be restricted to a closed block set; fills S.
int Session::try_closed(size_t s0, size_t s_edit, BlockSet &S) {
    const int beta = std::min(opts.block_bits, n_int);
    const uint64_t nblocks = uint64_t(1) << (n_int - beta);
    if (nblocks > (uint64_t(1) << 22)) return QTASK_E_UNSUPPORTED;
    // a state of one or two blocks gains nothing from a restricted replay,
    // which costs a tile-list upload and a wait
    if (nblocks < 4) return QTASK_E_UNSUPPORTED;
    const size_t nseg = segs_.size();
    if (s_edit >= nseg) return QTASK_E_UNSUPPORTED;
    // the segments after the edited one must be the same as at the last
    // update (same content, same anchors); match them from the end
    const size_t tail = nseg - s_edit;
    if (prev_hashes_.size() < tail) return QTASK_E_UNSUPPORTED;
    const size_t oe = prev_hashes_.size() - tail;
    for (size_t k = 1; k < tail; ++k)
        if (prev_hashes_[oe + k] != segs_[s_edit + k].hash) return QTASK_E_UNSUPPORTED;
    // and the segments from the restart point up to the edited one as well
    if (oe < s_edit - s0) return QTASK_E_UNSUPPORTED;
    for (size_t k = 1; k <= s_edit - s0; ++k)
        if (prev_hashes_[oe - k] != segs_[s_edit - k].hash) return QTASK_E_UNSUPPORTED;
    // the edited segment must start at the same boundary as the old one it
    // is compared with: removing the level that ended the previous segment
    // merges the two, and the old plan would then cover only part of the
    // new segment (a block rewritten only by the removed level would look
    // unchanged)
    if ((s_edit == 0) != (oe == 0)) return QTASK_E_UNSUPPORTED;
    if (s_edit > 0 && (prev_anchors_.size() != prev_hashes_.size() ||
                       prev_anchors_[oe - 1] != segs_[s_edit - 1].anchor))
        return QTASK_E_UNSUPPORTED;
    if (prev_hashes_[oe] == segs_[s_edit].hash) {
        S = BlockSet(nblocks);  // the edits cancelled out: nothing to redo
        return QTASK_OK;
    }
    auto old_it = plan_cache_.find(prev_hashes_[oe]);
    if (old_it == plan_cache_.end()) return QTASK_E_UNSUPPORTED;
    const auto &op = old_it->second.passes;
    const auto &np = plans_[s_edit]->passes;
    // Cheap lower bound first: the blocks rewritten by the gates that were
    // added or removed must be redone whatever else changed.  If even they
    // reach every block, the replay cannot be restricted.
    {
        auto gate_key = [](const LGate &g) {
            uint64_t id = hash_mix(1469598103934665603ull, g.kop);
            for (int q = 0; q < g.nq; ++q) id = hash_mix(id, uint64_t(g.q[q] + 1));
            return hash_mix(id, g.gate_id);
        };
        std::vector<std::pair<uint64_t, const LGate *>> a, b;
        for (const auto &p : op)
            for (const auto &stg : p.stages)
                for (const auto &g : stg.ops) a.emplace_back(gate_key(g), &g);
        for (const auto &p : np)
            for (const auto &stg : p.stages)
                for (const auto &g : stg.ops) b.emplace_back(gate_key(g), &g);
        auto by_key = [](const std::pair<uint64_t, const LGate *> &x, const std::pair<uint64_t, const LGate *> &y) {
            return x.first < y.first;
        };
        std::sort(a.begin(), a.end(), by_key);
        std::sort(b.begin(), b.end(), by_key);
        BlockSet lb(nblocks);
        size_t i = 0, j = 0;
        // an op of no controlled or phase form rewrites every block: the
        // bound is saturated at once (relabelling moves many ops to other
        // positions, and each would otherwise walk all blocks)
        bool sat = false;
        std::vector<const LGate *> diff;
        while (i < a.size() || j < b.size()) {
            if (j == b.size() || (i < a.size() && a[i].first < b[j].first)) diff.push_back(a[i++].second);
            else if (i == a.size() || b[j].first < a[i].first) diff.push_back(b[j++].second);
            else { ++i; ++j; }
        }
        for (const LGate *g : diff) sat = sat || rewrites_every_block(*g, beta);
        if (sat) return QTASK_E_UNSUPPORTED;
        // the bound walks every block per op: give up on the restriction
        // when that would cost more than planning a replay saves
        size_t actions = diff.size();
        for (size_t s = s_edit; s < nseg; ++s)
            for (const auto &p : plans_[s]->passes)
                for (const auto &stg : p.stages) actions += stg.U.empty() ? stg.ops.size() : 1;
        if (actions * nblocks > (uint64_t(1) << 28)) return QTASK_E_UNSUPPORTED;
        for (size_t k = 0; k < diff.size() && !sat; ++k)
            for_rewritten_blocks(*diff[k], beta, nblocks, [&](uint64_t blk) { lb.set(blk); });
        sat = sat || lb.all();
        for (size_t s = s_edit; s < nseg && !sat; ++s)
            for (const auto &p : plans_[s]->passes) {
                for_pass_actions(p, beta, [&](const BlockAction &ba) {
                    if (!sat) {
                        propagate(ba, lb);
                        sat = lb.all();
                    }
                });
                if (sat) break;
            }
        if (sat) return QTASK_E_UNSUPPORTED;
    }
    // Seeds: blocks whose ordered sequence of rewriting ops differs between
    // the old and the new plan of the edited segment.  A block rewritten by
    // the same ops in the same order from the same input ends with the same
    // bits unless another block feeds it, which the propagation below covers.
    size_t work = 0;
    for (const auto *ps : {&op, &np})
        for (const auto &p : *ps)
            for (const auto &stg : p.stages) work += stg.U.empty() ? stg.ops.size() : 1;
    if (work * nblocks > (uint64_t(1) << 28)) return QTASK_E_UNSUPPORTED;
    auto seq_hash = [&](const std::vector<PPass> &passes) {
        std::vector<uint64_t> h(nblocks, 0);
        auto mix = [&](uint64_t j, uint64_t v) { h[j] = hash_mix(h[j], v); };
        for (const auto &p : passes) {
            for (const auto &stg : p.stages) {
                if (!stg.U.empty()) {
                    uint64_t id = 1469598103934665603ull;
                    for (const cd &z : stg.U) id = hash_mix(hash_mix(id, double_bits(z.real())), double_bits(z.imag()));
                    for (int tb : stg.tbits) id = hash_mix(id, uint64_t(p.qlist[tb]));
                    for (uint64_t j = 0; j < nblocks; ++j) mix(j, id);
                    continue;
                }
                auto op_id = [&](const LGate &g) {
                    uint64_t id = hash_mix(1469598103934665603ull, g.kop);
                    for (int q = 0; q < g.nq; ++q) id = hash_mix(id, uint64_t(g.q[q] + 1));
                    for (const cd &z : g.m) id = hash_mix(hash_mix(id, double_bits(z.real())), double_bits(z.imag()));
                    return id;
                };
                for (const auto &g : stg.ops)
                    if (!lane_phase(p, stg, g)) {
                        const uint64_t id = op_id(g);
                        for_rewritten_blocks(g, beta, nblocks, [&](uint64_t j) { mix(j, id); });
                    }
                // the stage's lane phases come last, multiplied into one
                // factor per lane before it scales the registers: a block's
                // bits depend on which of them share a stage
                std::vector<uint64_t> hit;
                for (const auto &g : stg.ops)
                    if (lane_phase(p, stg, g)) {
                        const uint64_t id = hash_mix(op_id(g), 0x50454e44ull);
                        for_rewritten_blocks(g, beta, nblocks, [&](uint64_t j) {
                            mix(j, id);
                            hit.push_back(j);
                        });
                    }
                std::sort(hit.begin(), hit.end());
                hit.erase(std::unique(hit.begin(), hit.end()), hit.end());
                for (uint64_t j : hit) mix(j, 0x504849ull);
            }
            // a store permutation moves every amplitude of the tile's
            // positions: it counts as rewriting every block
            if (p.relabels()) {
                uint64_t id = hash_mix(0x52454c4142454cull, p.qlist.size());
                for (size_t k = 0; k < p.qlist.size(); ++k)
                    id = hash_mix(hash_mix(id, uint64_t(p.qlist[k])), uint64_t(p.out_pos(int(k))));
                for (uint64_t j = 0; j < nblocks; ++j) mix(j, id);
            }
        }
        return h;
    };
    const std::vector<uint64_t> ho = seq_hash(op), hn = seq_hash(np);
    BlockSet d(nblocks);
    for (uint64_t j = 0; j < nblocks; ++j)
        if (ho[j] != hn[j]) d.set(j);
    bool saturated = d.all();
    auto prop = [&](const PPass &p) {
        if (saturated) return;
        for_pass_actions(p, beta, [&](const BlockAction &ba) { propagate(ba, d); });
        saturated = d.all();
    };
    for (size_t i = 0; i < np.size(); ++i) prop(np[i]);
    for (size_t s = s_edit + 1; s < nseg; ++s)
        for (const auto &p : plans_[s]->passes) prop(p);
    if (saturated) return QTASK_E_UNSUPPORTED;
    // closedness over every replayed gate
    for (size_t s = s0; s < nseg; ++s)
        for (const auto &p : plans_[s]->passes) {
            bool ok = true;
            for_pass_actions(p, beta, [&](const BlockAction &ba) {
                if (ok && !closed_under(ba, d)) ok = false;
            });
            if (!ok) return QTASK_E_UNSUPPORTED;
        }
    S = d;
    return QTASK_OK;
}

// Host-only part of an update: segments, plans (kept on the host until the
// commit uploads them), the restart point, the closed-set decision and its
// tile lists, and the device bytes the session will hold after the commit.
// Nothing on the device changes here, so a failure (or a caller that decides
// not to commit) leaves the previous result and its checkpoints as they were.
int Session::plan_update(bool force_full) {
    const double t0 = now_ms();
    prep_t0_ = t0;
    prep_pending_ = false;
    prep_committed_ = false;
    launches.clear();
    qtask_stats st{};
    st.struct_size = sizeof(st);
    const size_t D = circ.num_levels();
    st.levels_total = D;
    st.total_blocks = uint64_t(1) << (n_int - std::min(opts.block_bits, n_int));
    prep_mode_ = 0;
    prep_tiles_.clear();
    prep_list_off_.clear();
    prep_need_bytes_ = device_bytes();

    PlanParams pp;
    pp.n = n_int;
    pp.b = std::min(opts.tile_bits, n_int);
    pp.c = std::min(opts.low_bits, pp.b);
    pp.dtype = dtype;
    pp.fusion = opts.fusion;
    pp.fuse_k = opts.fuse_width;
    pp.swz = dtype == QTASK_C128 ? 4 : 5;
    pp.relabel = opts.relabel;

    const bool full = force_full || !have_result_;
    if (!full && !circ.edited()) {
        st.plan_ms = now_ms() - t0;
        last = st;
        return QTASK_OK;  // mode 0: nothing to do
    }
    const size_t L = full ? 0 : circ.first_edited();
    prep_first_edit_ = L;

    // segments and their plans (cached by content)
    build_segments(pp);
    const size_t S = segs_.size();
    prep_S_ = S;
    plans_.assign(S, nullptr);
    // segments whose plan is not cached yet (one per distinct content);
    // plan_segment is a pure function, so they are planned concurrently
    std::vector<std::pair<uint64_t, std::vector<LGate>>> todo;
    for (size_t s = 0; s < S; ++s) {
        Seg &sg = segs_[s];
        auto kh = key_hash_.find(sg.key);
        if (kh != key_hash_.end() && plan_cache_.count(kh->second)) {
            sg.hash = kh->second;
            continue;
        }
        std::vector<LGate> ops = level_ops(sg.lo, sg.hi);
        sg.hash = segment_hash(ops, pp);
        key_hash_[sg.key] = sg.hash;
        if (plan_cache_.count(sg.hash)) continue;
        bool dup = false;
        for (const auto &td : todo) dup = dup || td.first == sg.hash;
        if (!dup) todo.emplace_back(sg.hash, std::move(ops));
    }
    constexpr size_t kPlanThreads = 8;
    for (size_t i0 = 0; i0 < todo.size(); i0 += kPlanThreads) {
        const size_t i1 = std::min(todo.size(), i0 + kPlanThreads);
        std::vector<std::future<SegmentPlan>> futs;
        for (size_t i = i0; i < i1; ++i)
            futs.push_back(std::async(i + 1 < i1 ? std::launch::async : std::launch::deferred,
                                      [&pp, &td = todo[i]] { return plan_segment(td.second, pp, td.first); }));
        for (size_t i = i0; i < i1; ++i) {
            try {
                plan_cache_.emplace(todo[i].first, futs[i - i0].get());
            } catch (const std::exception &e) {
                for (size_t j = i + 1; j < i1; ++j) futs[j - i0].wait();  // no thread outlives its inputs
                last_error = e.what();
                return QTASK_E_ARG;
            }
        }
    }
    for (size_t s = 0; s < S; ++s) plans_[s] = &plan_cache_.at(segs_[s].hash);

    // restart point: the newest valid checkpoint at or before the first
    // edited level (boundary j = the state before segment j)
    size_t s0 = 0, s_edit = 0;
    if (!full) {
        s_edit = S ? S - 1 : 0;
        for (size_t s = 0; s < S; ++s)
            if (segs_[s].hi > L) { s_edit = s; break; }
        auto usable = [&](size_t j) {
            auto it = ckpts_.find(segs_[j - 1].anchor);
            return stores_ckpt(j, S) && it != ckpts_.end() && it->second.valid && (plan_only || it->second.buf.p);
        };
        for (size_t j = s_edit; j >= 1; --j) {
            if (!usable(j) || segs_[j - 1].hi > L) continue;
            // a sparse restore reads the stored checkpoints before it as well
            bool chain = true;
            if (opts.ckpt_delta)
                for (size_t i = 1; i < j && chain; ++i) chain = !stores_ckpt(i, S) || usable(i);
            if (!chain) continue;
            s0 = j;
            break;
        }
    }
    for (size_t j = 1; j < S; ++j) (void)slot_of(segs_[j - 1].anchor);

    const bool renorm = dtype == QTASK_C64 && opts.renorm != 0;
    prep_renorm_ = renorm;
    int mode = full ? 1 : 2;
    BlockSet set;
    if (!full && opts.closed_mode && !renorm && S > 0 && !opts.ckpt_delta) {
        if (try_closed(s0, s_edit, set) == QTASK_OK) mode = 3;
    }
    // sparse checkpoints: what each boundary will hold, and how the restart
    // boundary's state is put together (when its own checkpoint holds only
    // some blocks): each block from the newest checkpoint at or before it
    // that holds the block, |0...0> where none does
    prep_restore_.clear();
    if (opts.ckpt_delta) {
        for (size_t s = 0; s + 1 < S; ++s) (void)written_blocks(*plans_[s]);
        if (s0 > 0) {
            const Ckpt &top = ckpts_.at(segs_[s0 - 1].anchor);
            if (!top.full) {
                const int beta = std::min(opts.block_bits, n_int);
                const uint64_t nblocks = uint64_t(1) << (n_int - beta);
                BlockSet done(nblocks);
                uint64_t left = nblocks;
                for (size_t j = s0; j >= 1 && left > 0; --j) {
                    if (!stores_ckpt(j, S)) continue;
                    const uint64_t a = segs_[j - 1].anchor;
                    const Ckpt &ck = ckpts_.at(a);
                    RestorePart part;
                    part.anchor = a;
                    if (ck.full) {
                        for (uint64_t b = 0; b < nblocks; ++b)
                            if (!done.test(b)) { part.dst.push_back(uint32_t(b)); part.src.push_back(uint32_t(b)); }
                        left = 0;
                    } else {
                        for (size_t k = 0; k < ck.blocks.size(); ++k)
                            if (!done.test(ck.blocks[k])) {
                                done.set(ck.blocks[k]);
                                part.dst.push_back(ck.blocks[k]);
                                part.src.push_back(uint32_t(k));
                                --left;
                            }
                    }
                    if (!part.dst.empty()) prep_restore_.push_back(std::move(part));
                }
                if (left > 0) {
                    RestorePart basis;
                    for (uint64_t b = 0; b < nblocks; ++b)
                        if (!done.test(b)) basis.dst.push_back(uint32_t(b));
                    prep_restore_.push_back(std::move(basis));
                }
            }
        }
    }
    prep_mode_ = mode;
    prep_s0_ = s0;
    st.mode = mode;
    st.first_level = S ? segs_[s0].lo : 0;
    st.segments_replayed = S - s0;
    st.levels_replayed = D - std::min(D, size_t(st.first_level));
    st.dirty_blocks = mode == 3 ? set.count() : st.total_blocks;
    if (mode == 3) prep_set_ = set;

    // tile lists for the closed replay
    if (mode == 3) {
        const int beta = std::min(opts.block_bits, n_int);
        const std::vector<uint32_t> blocks = set.list();
        for (size_t s = s0; s < S; ++s)
            for (size_t p = 0; p < plans_[s]->passes.size(); ++p) {
                const PPass &ps = plans_[s]->passes[p];
                const KPass &kp = reinterpret_cast<const KPass *>(plans_[s]->blob.data())[p];
                uint64_t nonq_low = 0;
                for (int q = 0; q < beta; ++q)
                    if (!((ps.qmask >> q) & 1)) nonq_low |= uint64_t(1) << q;
                std::vector<uint32_t> lows;
                // every combination of the non-pass bits below beta
                for (uint64_t sub = nonq_low;; sub = (sub - 1) & nonq_low) {
                    lows.push_back(uint32_t(sub));
                    if (sub == 0) break;
                }
                std::vector<uint32_t> tl;
                tl.reserve(blocks.size() * lows.size());
                for (uint32_t blk : blocks)
                    for (uint32_t lo : lows)
                        tl.push_back(uint32_t(pext_tile((uint64_t(blk) << beta) | lo, kp.nonq_pos, kp.n_nonq)));
                std::sort(tl.begin(), tl.end());
                tl.erase(std::unique(tl.begin(), tl.end()), tl.end());
                prep_list_off_.push_back(prep_tiles_.size());
                prep_tiles_.insert(prep_tiles_.end(), tl.begin(), tl.end());
            }
        prep_list_off_.push_back(prep_tiles_.size());
    }
    st.plan_ms = now_ms() - t0;
    last = st;
    prep_need_bytes_ = bytes_after_commit();
    prep_pending_ = true;
    return QTASK_OK;
}

// Sizes the commit grows the scratch buffers to (0: no growth needed).
Session::ScratchNeed Session::scratch_need() const {
    ScratchNeed z;
    const int b = std::min(opts.tile_bits, n_int);
    const size_t slots = next_slot_ + 1;
    if (scalars_cap_ / 2 < slots) z.scalars = 2 * std::max<size_t>(2 * slots, 64);
    const size_t np = std::max<size_t>(size_t(1) << (n_int - b), 4096);
    if (partials_cap_ < np) z.partials = np;
    if (!d_u64_ || u64_cap_ < 4096) z.u64 = 4096;
    if (prep_mode_ == 3) {
        if (tiles_cap_ < prep_tiles_.size()) z.tiles = prep_tiles_.size() + 4096;
        const size_t words = prep_set_.words().size();
        if (mask_cap_ < words) z.mask = words;
    }
    return z;
}

// Device bytes the session holds once the pending commit is done: the
// state, one buffer per stored checkpoint, the blobs of the plans in use and
// the scratch buffers (grown where the commit grows them).
uint64_t Session::bytes_after_commit() const {
    if (plan_only) return 0;
    if (!prep_pending_) return device_bytes();  // nothing planned: the commit changes nothing
    const size_t S = segs_.size();
    uint64_t b = state_bytes();
    for (size_t j = 1; j < S; ++j)
        if (stores_ckpt(j, S)) {
            const CkptLayout L = layout_of(j);
            b += L.bytes + (L.full ? 0 : L.blocks->size() * sizeof(uint32_t));
        }
    size_t restore = 0;
    for (const auto &part : prep_restore_) restore += part.dst.size() + part.src.size();
    b += std::max(restore, restore_cap_) * sizeof(uint32_t);
    std::unordered_set<uint64_t> live;
    for (const auto &sg : segs_)
        if (live.insert(sg.hash).second) b += plan_cache_.at(sg.hash).blob.size();
    const ScratchNeed z = scratch_need();
    b += (z.scalars ? z.scalars : scalars_cap_) * sizeof(double);
    b += (z.partials ? z.partials : partials_cap_) * sizeof(double);
    b += (z.u64 ? z.u64 : u64_cap_) * sizeof(unsigned long long);
    b += (z.tiles ? z.tiles : tiles_cap_) * sizeof(uint32_t);
    b += (z.mask ? z.mask : mask_cap_) * sizeof(uint64_t);
    return b;
}

// Device part of an update: allocate everything the planned replay needs
// first (plan blobs, checkpoint buffers, state, scratch), and only when all
// of it succeeded change the session's buffers, upload and build the launch
// list.  QTASK_E_NOMEM therefore leaves the previous result, its
// checkpoints and their validity untouched.
int Session::commit_device() {
    if (!prep_pending_) return QTASK_OK;
    if (prep_mode_ == 0) {
        prep_pending_ = false;
        return QTASK_OK;
    }
    const size_t S = prep_S_;
    const size_t s0 = prep_s0_;
    const int mode = prep_mode_;
    const bool renorm = prep_renorm_;
    qtask_stats &st = last;

    // --- 1. allocations (nothing of the session changes yet)
    std::vector<void *> fresh;
    auto undo = [&] {
        for (void *p : fresh) dfree(p);
        return QTASK_E_NOMEM;
    };
    auto grab = [&](size_t bytes) {
        void *p = dalloc(bytes);
        if (p) fresh.push_back(p);
        return p;
    };
    std::vector<std::pair<SegmentPlan *, void *>> plan_bufs;
    struct CkNew {
        uint64_t anchor;
        CkptLayout L;
        void *buf = nullptr, *dbl = nullptr;
        uint64_t spare = 0;  // take the buffer of this boundary (no longer stored)
    };
    std::vector<CkNew> cknew;          // stored boundaries that need a (new) buffer
    std::vector<uint64_t> spare_ckpt;  // whole-state buffers of boundaries no longer stored
    std::unordered_set<uint64_t> stored;
    size_t restore_need = 0;
    uint32_t *new_restore = nullptr;
    void *new_state = nullptr;
    double *new_scalars = nullptr, *new_partials = nullptr;
    unsigned long long *new_u64 = nullptr;
    uint32_t *new_tiles = nullptr;
    uint64_t *new_mask = nullptr;
    const ScratchNeed z = scratch_need();
    if (!plan_only) {
        std::unordered_set<uint64_t> seen;
        for (const auto &sg : segs_) {
            SegmentPlan &sp = plan_cache_.at(sg.hash);
            if (sp.dev || !seen.insert(sg.hash).second) continue;
            void *p = grab(sp.blob.size());
            if (!p) return undo();
            plan_bufs.emplace_back(&sp, p);
        }
        // checkpoints: a new buffer wherever a stored boundary has none or
        // needs another layout (sparse checkpoints follow their segment's
        // plan); whole-state buffers of boundaries no longer stored are
        // reused first
        for (size_t j = 1; j < S; ++j) {
            if (!stores_ckpt(j, S)) continue;
            const uint64_t a = segs_[j - 1].anchor;
            stored.insert(a);
            const CkptLayout L = layout_of(j);
            auto it = ckpts_.find(a);
            if (it == ckpts_.end() || !it->second.buf.p || it->second.wkey != L.wkey) cknew.push_back({a, L});
        }
        for (const auto &kv : ckpts_)
            if (!stored.count(kv.first) && kv.second.buf.p && kv.second.full) spare_ckpt.push_back(kv.first);
        size_t nspare = 0;
        for (auto &cn : cknew) {
            if (cn.L.full && nspare < spare_ckpt.size()) {
                cn.spare = spare_ckpt[nspare++];
                continue;
            }
            if (!(cn.buf = grab(cn.L.bytes))) return undo();
            if (!cn.L.full && !(cn.dbl = grab(cn.L.blocks->size() * sizeof(uint32_t)))) return undo();
        }
        for (const auto &part : prep_restore_) restore_need += part.dst.size() + part.src.size();
        if (restore_need > restore_cap_ &&
            !(new_restore = static_cast<uint32_t *>(grab(restore_need * sizeof(uint32_t)))))
            return undo();
        if (!state_.p && !(new_state = grab(state_bytes()))) return undo();
        if (z.scalars && !(new_scalars = static_cast<double *>(grab(z.scalars * sizeof(double))))) return undo();
        if (z.partials && !(new_partials = static_cast<double *>(grab(z.partials * sizeof(double))))) return undo();
        if (z.u64 && !(new_u64 = static_cast<unsigned long long *>(grab(z.u64 * sizeof(unsigned long long)))))
            return undo();
        if (z.tiles && !(new_tiles = static_cast<uint32_t *>(grab(z.tiles * sizeof(uint32_t))))) return undo();
        if (z.mask && !(new_mask = static_cast<uint64_t *>(grab(z.mask * sizeof(uint64_t))))) return undo();
    }

    // --- 2. commit: from here on only device errors can fail
    prep_pending_ = false;
    prep_committed_ = true;
    if (!plan_only) {
        for (auto &pb : plan_bufs) {
            pb.first->dev = pb.second;
            pb.first->dev_bytes = pb.first->blob.size();
            HIPCHK(hipMemcpyAsync(pb.second, pb.first->blob.data(), pb.first->blob.size(), hipMemcpyHostToDevice,
                                  stream));
        }
        std::vector<void *> drop;  // buffers replaced by another layout
        for (auto &cn : cknew) {
            Ckpt &ck = ckpts_[cn.anchor];
            drop.push_back(ck.buf.p);
            drop.push_back(ck.d_blocks.p);
            if (cn.spare) {
                Ckpt &old = ckpts_.at(cn.spare);
                ck.buf = old.buf;
                old.buf = DevBuf{};
            } else {
                ck.buf = DevBuf{cn.buf, size_t(cn.L.bytes)};
            }
            ck.full = cn.L.full;
            ck.wkey = cn.L.wkey;
            ck.blocks = cn.L.full ? std::vector<uint32_t>() : *cn.L.blocks;
            ck.d_blocks = cn.L.full ? DevBuf{} : DevBuf{cn.dbl, ck.blocks.size() * sizeof(uint32_t)};
            if (!ck.blocks.empty())
                HIPCHK(hipMemcpyAsync(ck.d_blocks.p, ck.blocks.data(), ck.d_blocks.bytes, hipMemcpyHostToDevice,
                                      stream));
            ck.valid = false;
        }
        for (auto it = ckpts_.begin(); it != ckpts_.end();) {
            if (!stored.count(it->first)) {
                dfree(it->second.buf.p);
                dfree(it->second.d_blocks.p);
                it = ckpts_.erase(it);
            } else {
                ++it;
            }
        }
        if (new_restore) {
            dfree(d_restore_);
            d_restore_ = new_restore;
            restore_cap_ = restore_need;
        }
        if (!prep_restore_.empty()) {
            size_t off = 0;
            for (const auto &part : prep_restore_) {
                HIPCHK(hipMemcpyAsync(d_restore_ + off, part.dst.data(), part.dst.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, stream));
                off += part.dst.size();
                if (!part.src.empty())
                    HIPCHK(hipMemcpyAsync(d_restore_ + off, part.src.data(), part.src.size() * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, stream));
                off += part.src.size();
            }
        }
        HIPCHK(hipStreamSynchronize(stream));  // the block lists are pageable host memory
        for (void *p : drop) dfree(p);
        if (new_state) {
            state_.p = new_state;
            state_.bytes = state_bytes();
        }
        if (new_scalars) {
            const size_t half = z.scalars / 2;
            if (d_scalars_) {
                // keep the norms and scales of still-valid checkpoints
                const size_t old = scalars_cap_ / 2;
                HIPCHK(hipMemcpyAsync(new_scalars, d_scalars_, old * sizeof(double), hipMemcpyDeviceToDevice, stream));
                HIPCHK(hipMemcpyAsync(new_scalars + half, d_scalars_ + old, old * sizeof(double),
                                      hipMemcpyDeviceToDevice, stream));
                HIPCHK(hipStreamSynchronize(stream));
                dfree(d_scalars_);
            }
            d_scalars_ = new_scalars;
            scalars_cap_ = z.scalars;
        }
        if (new_partials) {
            dfree(d_partials_);
            d_partials_ = new_partials;
            partials_cap_ = z.partials;
        }
        if (new_u64) {
            dfree(d_u64_);
            d_u64_ = new_u64;
            u64_cap_ = z.u64;
        }
        if (new_tiles) {
            dfree(d_tiles_);
            d_tiles_ = new_tiles;
            tiles_cap_ = z.tiles;
        }
        if (new_mask) {
            dfree(d_mask_);
            d_mask_ = new_mask;
            mask_cap_ = z.mask;
        }
        if (mode == 3) {
            if (!prep_tiles_.empty())
                HIPCHK(hipMemcpyAsync(d_tiles_, prep_tiles_.data(), prep_tiles_.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, stream));
            const auto &w = prep_set_.words();
            HIPCHK(hipMemcpyAsync(d_mask_, w.data(), w.size() * sizeof(uint64_t), hipMemcpyHostToDevice, stream));
            // pageable copies: make sure they completed before the host vectors change
            HIPCHK(hipStreamSynchronize(stream));
        }
    } else {
        // plan-only sessions keep a record per stored boundary (no buffers)
        for (auto it = ckpts_.begin(); it != ckpts_.end();) {
            bool keep = false;
            for (size_t j = 1; j < S && !keep; ++j)
                keep = segs_[j - 1].anchor == it->first && stores_ckpt(j, S);
            it = keep ? std::next(it) : ckpts_.erase(it);
        }
        for (size_t j = 1; j < S; ++j)
            if (stores_ckpt(j, S)) {
                const CkptLayout L = layout_of(j);
                Ckpt &ck = ckpts_[segs_[j - 1].anchor];
                if (ck.wkey != L.wkey) ck.valid = false;
                ck.full = L.full;
                ck.wkey = L.wkey;
                ck.blocks = L.full ? std::vector<uint32_t>() : *L.blocks;
            }
    }

    // launch list
    size_t li = 0;
    double bytes = 0, flops = 0, mfma_flops = 0;
    double *scales = plan_only ? nullptr : d_scalars_ + scalars_cap_ / 2;
    st.passes = st.stages = st.tiles = st.gate_amp_updates = 0;
    const int beta = std::min(opts.block_bits, n_int);
    const double block_bytes = double(uint64_t(1) << beta) * double(elem);
    // a sparse restore first puts the restart boundary's state together in
    // the state buffer, block by block from the checkpoints that hold it
    {
        size_t off = 0;
        for (const auto &part : prep_restore_) {
            Launch L{};
            L.kind = 1;
            L.cdst = state_.p;
            L.csrc = part.anchor && !plan_only ? ckpts_.at(part.anchor).buf.p : nullptr;
            L.cdst_idx = plan_only ? nullptr : d_restore_ + off;
            off += part.dst.size();
            L.csrc_idx = part.src.empty() || plan_only ? nullptr : d_restore_ + off;
            off += part.src.size();
            L.cn = uint32_t(part.dst.size());
            L.b = beta;
            launches.push_back(L);
            bytes += double(part.dst.size()) * block_bytes * (part.anchor ? 2 : 1);
        }
    }
    for (size_t s = s0; s < S; ++s) {
        const SegmentPlan &sp = *plans_[s];
        const int b = sp.pp.b;
        const uint64_t full_tiles = uint64_t(1) << (n_int - b);
        const char *blob = static_cast<const char *>(sp.dev);
        const size_t P = sp.passes.size();
        const size_t end_slot = s + 1 < S ? slot_of(segs_[s].anchor) : 0;
        void *end_ckpt = nullptr;
        const Ckpt *end_ck = nullptr;
        if (s + 1 < S && stores_ckpt(s + 1, S)) {
            end_ck = &ckpts_.at(segs_[s].anchor);
            if (!plan_only && end_ck->full) end_ckpt = end_ck->buf.p;  // a whole copy rides on the last pass
        }
        for (size_t p = 0; p < P; ++p, ++li) {
            Launch L{};
            KArgs &a = L.args;
            a.dst = state_.p;
            if (s == s0 && p == 0) {
                if (!prep_restore_.empty()) a.src = state_.p;  // put together in place above
                else if (s0 == 0) { a.src_basis = 1; a.src = nullptr; }
                else a.src = plan_only ? nullptr : ckpts_.at(segs_[s0 - 1].anchor).buf.p;
            } else {
                a.src = state_.p;
            }
            const bool lastp = p + 1 == P;
            a.scale = (renorm && p == 0 && s > 0 && !plan_only) ? scales + slot_of(segs_[s - 1].anchor) : nullptr;
            a.ckpt = lastp ? end_ckpt : nullptr;
            a.partials = (lastp && renorm) ? d_partials_ : nullptr;
            a.pass = reinterpret_cast<const KPass *>(blob) + p;
            a.stages = reinterpret_cast<const KStage *>(blob + sp.off_stage);
            a.ops = reinterpret_cast<const KOp *>(blob + sp.off_op);
            a.coefs = blob + sp.off_coef;
            a.block_bits = uint32_t(std::min(opts.block_bits, n_int));
            a.has_mfma = sp.passes[p].has_mfma ? 1 : 0;
            a.has_dense = sp.passes[p].has_dense ? 1 : 0;
            uint64_t tiles = full_tiles;
            if (mode == 3) {
                tiles = prep_list_off_[li + 1] - prep_list_off_[li];
                a.tile_list = d_tiles_ ? d_tiles_ + prep_list_off_[li] : nullptr;
                a.store_mask = d_mask_;
            }
            L.n_tiles = uint32_t(tiles);
            L.b = b;
            L.after = (lastp && renorm) ? 1 : 0;
            L.slot = end_slot;
            if (tiles > 0 || L.after) launches.push_back(L);
            const double tb = double(uint64_t(1) << b) * double(elem);
            bytes += double(tiles) * tb * ((a.src_basis ? 0 : 1) + 1 + (a.ckpt ? 1 : 0));
            double pf = 0, mf = 0;
            for (const auto &stg : sp.passes[p].stages) {
                pf += stg.flops;
                if (stg.mfma) mf += stg.flops;
            }
            flops += double(tiles) * double(uint64_t(1) << b) * pf;
            mfma_flops += double(tiles) * double(uint64_t(1) << b) * mf;
            if (tiles > 0) {
                st.passes += 1;
                st.stages += sp.passes[p].stages.size();
            }
            st.tiles += tiles;
        }
        if (end_ck && !end_ck->full) {
            // a sparse checkpoint: its blocks are copied out after the segment
            Launch L{};
            L.kind = 1;
            L.cdst = plan_only ? nullptr : end_ck->buf.p;
            L.csrc = state_.p;
            L.csrc_idx = static_cast<const uint32_t *>(end_ck->d_blocks.p);
            L.cn = uint32_t(end_ck->blocks.size());
            L.b = beta;
            launches.push_back(L);
            bytes += 2.0 * double(end_ck->blocks.size()) * block_bytes;
        }
        st.gate_amp_updates += sp.n_gates * (uint64_t(1) << n);
    }
    st.ckpt_bytes = st.ckpt_full_bytes = 0;
    for (size_t j = 1; j < S; ++j)
        if (stores_ckpt(j, S)) {
            const Ckpt &ck = ckpts_.at(segs_[j - 1].anchor);
            st.ckpt_bytes += ck.full ? state_bytes() : uint64_t(ck.blocks.size()) * (uint64_t(1) << beta) * elem;
            st.ckpt_full_bytes += state_bytes();
        }
    if (renorm && S > 0) bytes += 2.0 * double(state_bytes());
    st.bytes = bytes;
    st.flops = flops;
    st.mfma_flops = mfma_flops;
    // drop cached plans no segment uses any more
    {
        std::unordered_set<uint64_t> live;
        for (const auto &sg : segs_) live.insert(sg.hash);
        for (auto it = plan_cache_.begin(); it != plan_cache_.end();) {
            if (!live.count(it->first)) {
                dfree(it->second.dev);
                it = plan_cache_.erase(it);
            } else {
                ++it;
            }
        }
        for (auto it = key_hash_.begin(); it != key_hash_.end();)
            it = live.count(it->second) ? std::next(it) : key_hash_.erase(it);
    }
    st.plan_ms = now_ms() - prep_t0_;
    return QTASK_OK;
}

int Session::prepare(bool force_full) {
    int rc = plan_update(force_full);
    if (rc != QTASK_OK) return rc;
    return commit_device();
}

int Session::enqueue_after(const Launch &L, hipStream_t s) {
    if (L.after == 1) {
        double *norms = d_scalars_;
        double *scales = d_scalars_ + scalars_cap_ / 2;
        HIPCHK(launch_sum_partials(d_partials_, L.n_tiles, norms + L.slot, scales + L.slot, s));
    }
    return QTASK_OK;
}

int Session::enqueue_final(hipStream_t s) {
    if (prep_S_ == 0) {
        HIPCHK(launch_fill_basis(dtype, state_.p, uint64_t(1) << n_int, s));
    } else if (prep_renorm_ && prep_mode_ != 0) {
        // slot 0 holds the scale computed at the end of the circuit
        HIPCHK(launch_scale(dtype, state_.p, uint64_t(1) << n_int, d_scalars_ + scalars_cap_ / 2, s));
    }
    return QTASK_OK;
}

int Session::enqueue_prepared(hipStream_t s) {
    for (const Launch &L : launches) {
        if (L.kind == 1) {
            HIPCHK(launch_block_copy(dtype, L.cdst, L.csrc, L.cdst_idx, L.csrc_idx, L.cn, L.b, s));
            continue;
        }
        if (L.n_tiles > 0) HIPCHK(launch_pass(dtype, L.args, L.n_tiles, L.b, s));
        int rc = enqueue_after(L, s);
        if (rc != QTASK_OK) return rc;
    }
    return enqueue_final(s);
}

int Session::finish_prepared_host() {
    if (prep_mode_ == 0 || !prep_committed_) return QTASK_OK;
    prep_committed_ = false;
    const size_t S = prep_S_;
    for (size_t j = 1; j < S; ++j) {
        auto it = ckpts_.find(segs_[j - 1].anchor);
        if (it == ckpts_.end()) continue;
        // j > s0: rewritten by this replay -- wholly in modes 1 and 2; in
        // mode 3 only the affected blocks were stored, which keeps a valid
        // checkpoint valid (its other blocks are unchanged) and cannot make
        // an invalid one valid.  j <= s0: unchanged, valid if it was.
        if (j > prep_s0_ && prep_mode_ != 3) it->second.valid = true;
    }
    prev_hashes_.clear();
    prev_anchors_.clear();
    for (const auto &sg : segs_) {
        prev_hashes_.push_back(sg.hash);
        prev_anchors_.push_back(sg.anchor);
    }
    circ.clear_edits();
    have_result_ = true;
    state_valid_ = !plan_only;
    return QTASK_OK;
}

void Session::invalidate() {
    state_valid_ = false;
    have_result_ = false;
    for (auto &kv : ckpts_) kv.second.valid = false;
}

int Session::ensure_tuned() {
    if (!opts.autotune || tuned_ || plan_only) return QTASK_OK;
    const int rc = autotune();
    if (rc == QTASK_OK) tuned_ = true;
    return rc;
}

int Session::update(bool force_full) {
    const double t0 = now_ms();
    int rc = init_device();
    if (rc != QTASK_OK) return rc;
    rc = ensure_tuned();
    if (rc != QTASK_OK) return rc;
    rc = plan_update(force_full);
    if (rc == QTASK_OK) rc = commit_device();
    if (rc == QTASK_E_DEVICE) invalidate();
    if (rc != QTASK_OK) return rc;  // planning and allocation failures keep the previous result
    if (prep_mode_ == 0) {
        last.wall_ms = now_ms() - t0;
        return QTASK_OK;
    }
    if (!plan_only) {
        auto fail = [&](int code) {
            invalidate();
            return code;
        };
        if (hipEventRecord(ev0_, stream) != hipSuccess) return fail(QTASK_E_DEVICE);
        rc = enqueue_prepared(stream);
        if (rc != QTASK_OK) {
            (void)hipStreamSynchronize(stream);
            return fail(rc);
        }
        if (hipEventRecord(ev1_, stream) != hipSuccess) return fail(QTASK_E_DEVICE);
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            last_error = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
            return fail(QTASK_E_DEVICE);
        }
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev0_, ev1_) == hipSuccess) {
            last.kernel_ms = ms;
            last.pass_kernel_ms = ms;
        }
    }
    finish_prepared_host();
    last.wall_ms = now_ms() - t0;
    return QTASK_OK;
}

void Session::release_device() {
    if (plan_only) return;
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto &kv : plan_cache_) dfree(kv.second.dev);
    plan_cache_.clear();
    key_hash_.clear();
    plans_.clear();
    prev_hashes_.clear();
    prev_anchors_.clear();
    for (auto &kv : ckpts_) dfree(kv.second.buf.p);
    ckpts_.clear();
    dfree(state_.p);
    state_ = DevBuf{};
    dfree(d_partials_); d_partials_ = nullptr; partials_cap_ = 0;
    dfree(d_scalars_); d_scalars_ = nullptr; scalars_cap_ = 0;
    dfree(d_u64_); d_u64_ = nullptr; u64_cap_ = 0;
    dfree(d_mask_); d_mask_ = nullptr; mask_cap_ = 0;
    dfree(d_tiles_); d_tiles_ = nullptr; tiles_cap_ = 0;
    state_valid_ = false;
    have_result_ = false;
}

int Session::read(uint64_t first, uint64_t count, void *out) {
    if (plan_only) return QTASK_E_UNSUPPORTED;
    if (!state_valid_ || !state_.p || circ.edited()) return QTASK_E_STALE;
    const uint64_t N = uint64_t(1) << n;
    if (first > N || count > N - first) return QTASK_E_NOTFOUND;
    if (count == 0) return QTASK_OK;
    if (!out) return QTASK_E_ARG;
    HIPCHK(hipSetDevice(opts.device));
    HIPCHK(hipMemcpyAsync(out, static_cast<char *>(state_.p) + first * elem, count * elem, hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
    return QTASK_OK;
}

int Session::norm(double *out) {
    if (plan_only) return QTASK_E_UNSUPPORTED;
    if (!state_valid_ || !state_.p || circ.edited()) return QTASK_E_STALE;
    HIPCHK(hipSetDevice(opts.device));
    const uint64_t N = uint64_t(1) << n_int;
    HIPCHK(launch_norm(dtype, state_.p, N, d_partials_, reinterpret_cast<double *>(d_u64_), nullptr, stream));
    double v = 0;
    HIPCHK(hipMemcpyAsync(&v, d_u64_, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *out = v;
    return QTASK_OK;
}

int Session::hash(uint64_t *out) {
    if (plan_only) return QTASK_E_UNSUPPORTED;
    if (!state_valid_ || !state_.p || circ.edited()) return QTASK_E_STALE;
    HIPCHK(hipSetDevice(opts.device));
    const uint64_t N = uint64_t(1) << n_int;
    HIPCHK(launch_hash(dtype, state_.p, N, d_u64_ + 1, d_u64_, stream));
    unsigned long long v = 0;
    HIPCHK(hipMemcpyAsync(&v, d_u64_, sizeof(v), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *out = v;
    return QTASK_OK;
}

// Graphviz form of the plan: one cluster per segment (its level range), one
// node per pass in execution order (its tile qubits and, per stage, the
// register qubits and op count), edges in execution order; an edge that
// crosses a segment boundary says whether a checkpoint is stored there.
std::string Session::plan_dot() const {
    std::ostringstream o;
    o << "digraph qtask {\n  rankdir=LR;\n  node [shape=box, fontname=\"monospace\"];\n";
    std::vector<std::string> nodes;
    std::vector<size_t> seg_of;
    const size_t S = std::min(segs_.size(), plans_.size());
    for (size_t s = 0; s < S; ++s) {
        o << "  subgraph cluster_s" << s << " {\n    label=\"segment " << s << ": levels [" << segs_[s].lo << ", "
          << segs_[s].hi << ")\";\n";
        const auto &passes = plans_[s]->passes;
        for (size_t p = 0; p < passes.size(); ++p) {
            const std::string id = "p" + std::to_string(s) + "_" + std::to_string(p);
            o << "    " << id << " [label=\"pass " << p << "\\lqubits";
            for (int q : passes[p].qlist) o << " " << q;
            o << "\\l";
            for (const auto &st : passes[p].stages) {
                o << (st.mfma ? "mfma" : !st.U.empty() ? "dense" : "stage") << " {";
                for (size_t i = 0; i < st.tbits.size(); ++i) o << (i ? " " : "") << passes[p].qlist[st.tbits[i]];
                o << "}: " << st.ops.size() << " ops\\l";
            }
            o << "\"];\n";
            nodes.push_back(id);
            seg_of.push_back(s);
        }
        o << "  }\n";
    }
    for (size_t i = 1; i < nodes.size(); ++i) {
        o << "  " << nodes[i - 1] << " -> " << nodes[i];
        if (seg_of[i] != seg_of[i - 1])
            o << " [label=\"" << (stores_ckpt(seg_of[i], S) ? "checkpoint" : "boundary") << "\", style=bold]";
        o << ";\n";
    }
    o << "}\n";
    return o.str();
}

int Session::dump(const char *path) {
    const size_t len = std::strlen(path);
    if (len >= 4 && std::strcmp(path + len - 4, ".dot") == 0) {
        FILE *f = std::fopen(path, "w");
        if (!f) return QTASK_E_ARG;
        const std::string dot = plan_dot();
        const size_t wr = std::fwrite(dot.data(), 1, dot.size(), f);
        std::fclose(f);
        return wr == dot.size() ? QTASK_OK : QTASK_E_ARG;
    }
    std::ostringstream o;
    o << "{\"n\":" << n << ",\"n_buffer\":" << n_int << ",\"dtype\":" << dtype << ",\"levels\":" << circ.num_levels()
      << ",\"gates\":" << circ.num_gates() << ",\"tile_bits\":" << opts.tile_bits << ",\"low_bits\":" << opts.low_bits
      << ",\"block_bits\":" << std::min(opts.block_bits, n_int) << ",\"ckpt_interval\":" << opts.ckpt_interval
      << ",\"last\":{\"mode\":" << last.mode << ",\"first_level\":" << last.first_level
      << ",\"segments_replayed\":" << last.segments_replayed << ",\"passes\":" << last.passes
      << ",\"tiles\":" << last.tiles << ",\"dirty_blocks\":" << last.dirty_blocks
      << ",\"total_blocks\":" << last.total_blocks << "}";
    o << ",\"dirty_block_list\":[";
    if (last.mode == 3) {
        const auto l = prep_set_.list();
        for (size_t i = 0; i < l.size() && i < 65536; ++i) o << (i ? "," : "") << l[i];
    }
    o << "],\"checkpoints\":[";
    {
        bool firstc = true;
        for (size_t j = 1; j < segs_.size(); ++j) {
            if (!stores_ckpt(j, segs_.size())) continue;
            auto it = ckpts_.find(segs_[j - 1].anchor);
            if (it == ckpts_.end()) continue;
            o << (firstc ? "" : ",") << "{\"boundary\":" << j << ",\"level\":" << segs_[j - 1].hi
              << ",\"valid\":" << (it->second.valid ? "true" : "false") << ",\"full\":"
              << (it->second.full ? "true" : "false") << ",\"blocks\":[";
            for (size_t k = 0; k < it->second.blocks.size(); ++k) o << (k ? "," : "") << it->second.blocks[k];
            o << "]}";
            firstc = false;
        }
    }
    o << "],\"segments\":[";
    for (size_t s = 0; s < plans_.size(); ++s) {
        if (s) o << ",";
        o << plan_json(*plans_[s], true);
    }
    o << "]}";
    FILE *f = std::fopen(path, "w");
    if (!f) return QTASK_E_ARG;
    const std::string js = o.str();
    const size_t wr = std::fwrite(js.data(), 1, js.size(), f);
    std::fclose(f);
    return wr == js.size() ? QTASK_OK : QTASK_E_ARG;
}

}  // namespace qtask
