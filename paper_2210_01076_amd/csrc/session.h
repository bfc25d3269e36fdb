// One simulation handle: circuit store, segment plans, device state and
// checkpoints, and the full / incremental update.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/qtask.h"
#include "circuit.h"
#include "kdefs.h"
#include "planner.h"
#include "tracker.h"

namespace qtask {

double now_ms();

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

class Session {
public:
    Session(int n, int dtype, const qtask_opts &opts);
    ~Session();

    Circuit circ;
    int n;          // user qubits
    int n_int;      // qubits of the buffer (>= QK_MIN_TILE_BITS)
    int dtype;
    size_t elem;    // bytes per amplitude
    qtask_opts opts;
    bool plan_only;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    int init_device();   // called lazily; creates stream, scratch
    int autotune();      // picks opts.tile_bits / opts.low_bits by timing (first update)
    int ensure_tuned();  // autotune() once, when opts.autotune asks for it
    // forget the state and every checkpoint (after a failed replay): the
    // next update re-simulates from the start
    void invalidate();
    int update(bool force_full);
    int read(uint64_t first, uint64_t count, void *out);
    int norm(double *out);
    int hash(uint64_t *out);
    std::string plan_dot() const;
    int dump(const char *path);
    uint64_t device_bytes() const;
    uint64_t state_bytes() const { return (uint64_t(1) << n_int) * elem; }
    // bytes this session needs resident for its current circuit (state,
    // checkpoints, plans); used for admission
    uint64_t planned_bytes() const;

    // --- an update in two phases (also used by the server): plan_update()
    // runs on the host only (segments, plans, restart point, closed-set
    // decision) and leaves the device untouched; commit_device() allocates
    // everything the replay needs before it changes any buffer, then uploads
    // and builds the launch list.  A failure in either keeps the previous
    // result and its checkpoints.
    int plan_update(bool force_full);
    int commit_device();
    // device bytes held after the pending commit (valid after plan_update)
    uint64_t bytes_after_commit() const;
    // the circuit (and its segment cut) before a batch of modifiers, so that
    // a request whose edits or update fail can be undone as a whole
    void save_edit_point() { saved_circ_ = circ; saved_anchors_ = anchors_; }
    void rollback_edit_point() {
        circ = saved_circ_;
        anchors_ = saved_anchors_;
        prep_pending_ = false;
        prep_committed_ = false;
        launches.clear();
    }
    int prepare(bool force_full);           // plan_update + commit_device (no launches)
    struct Launch {                          // one launch of the prepared replay
        KArgs args;
        uint32_t n_tiles;
        int b;
        int after;          // 0 none, 1 sum partials -> norm and renorm scale of `slot`
        size_t slot;
        int kind = 0;       // 0 pass; 1 block copy (sparse checkpoint capture or restore)
        void *cdst = nullptr;
        const void *csrc = nullptr;
        const uint32_t *cdst_idx = nullptr, *csrc_idx = nullptr;
        uint32_t cn = 0;
    };
    std::vector<Launch> launches;            // filled by prepare()
    int finish_prepared_host();             // bookkeeping after the launches ran
    int enqueue_prepared(hipStream_t s);     // launch everything prepare() built
    int enqueue_after(const Launch &l, hipStream_t s);  // the tail work of a launch (renorm sums)
    int enqueue_final(hipStream_t s);        // work after the last pass (final renorm, empty circuit)

    // free every device buffer (state, checkpoints, plans, scratch); the next
    // update re-simulates from scratch
    void release_device();
    void release_state() {
        dfree(state_.p);
        state_ = DevBuf{};
    }
    // where the renormalisation sum of a launch with after == 1 goes
    void sum_targets(const Launch &l, const double **partials, double **norm, double **scale) const {
        *partials = d_partials_;
        *norm = d_scalars_ + l.slot;
        *scale = d_scalars_ + scalars_cap_ / 2 + l.slot;
    }
    int prep_mode() const { return prep_mode_; }
    bool needs_final() const { return prep_S_ == 0 || (prep_renorm_ && prep_mode_ != 0); }

    void *state() const { return state_.p; }
    bool state_valid() const { return state_valid_ && state_.p != nullptr; }
    qtask_stats last{};
    std::string last_error;

    void *dalloc(size_t bytes);
    void dfree(void *p);

private:
    // A segment is a run of levels [lo, hi) that ends at an anchor level (the
    // last segment ends at the end of the circuit).  Anchors are level ids:
    // inserting a level only grows the segment it lands in, so the plans and
    // checkpoints of the other segments stay usable.
    struct Seg {
        size_t lo = 0, hi = 0;
        uint64_t anchor = 0;   // id of level hi-1
        uint64_t key = 0;      // ids and versions of the segment's levels
        uint64_t hash = 0;     // content hash (plan cache key)
    };
    // A checkpoint holds the state at a segment boundary: the whole state,
    // or (sparse checkpoints) only the blocks the segment before it can
    // change, packed in the order of `blocks` (the others are as at the
    // previous boundary).
    struct Ckpt {
        DevBuf buf;
        bool valid = false;
        bool full = true;
        uint64_t wkey = 0;             // identifies the block list (0: whole state)
        std::vector<uint32_t> blocks;  // sparse: the blocks held, in buffer order
        DevBuf d_blocks;               // sparse: the same list on the device
    };
    // Layout a boundary's checkpoint gets from the plan of the segment
    // before it (the whole state unless sparse checkpoints are on and the
    // segment changes only some blocks).
    struct CkptLayout {
        bool full = true;
        uint64_t wkey = 0;
        const std::vector<uint32_t> *blocks = nullptr;
        uint64_t bytes = 0;
    };
    CkptLayout layout_of(size_t j) const;
    const std::vector<uint32_t> &written_blocks(const SegmentPlan &sp);
    std::unordered_map<uint64_t, std::vector<uint32_t>> wsets_;  // plan hash -> blocks it can change (empty: all)
    // unions of consecutive segments' block sets (a stored boundary after
    // boundaries that are not stored), by a key of the segments' set keys
    mutable std::unordered_map<uint64_t, std::vector<uint32_t>> unions_;
    std::unordered_map<uint64_t, uint64_t> wkeys_;               // plan hash -> key of that list
    int K() const { return opts.ckpt_interval; }
    size_t num_segments() const { return (circ.num_levels() + size_t(K()) - 1) / size_t(K()); }
    bool stores_ckpt(size_t j, size_t S) const;
    std::vector<LGate> level_ops(size_t lo, size_t hi) const;
    void build_segments(const PlanParams &pp);
    size_t slot_of(uint64_t anchor);
    int ensure_state();
    int upload_plan(SegmentPlan &sp);
    int try_closed(size_t s0, size_t s_edit, BlockSet &S);

    DevBuf state_;
    std::vector<Seg> segs_;
    std::vector<SegmentPlan *> plans_;                    // plan of segs_[s]
    std::unordered_map<uint64_t, SegmentPlan> plan_cache_;  // by content hash
    std::unordered_map<uint64_t, uint64_t> key_hash_;       // segment key -> content hash
    // lowered gates by gate id (ids are never reused; lowering is a pure
    // function of kind, qubits and parameters); pruned when it outgrows the
    // circuit
    mutable std::unordered_map<uint64_t, LGate> lowered_;
    std::vector<uint64_t> prev_hashes_;                   // segment hashes at the last update
    std::vector<uint64_t> prev_anchors_;                  // segment end anchors at the last update
    std::unordered_set<uint64_t> anchors_;
    Circuit saved_circ_{0};
    std::unordered_set<uint64_t> saved_anchors_;
    std::unordered_map<uint64_t, Ckpt> ckpts_;            // by anchor level id
    std::unordered_map<uint64_t, size_t> slots_;          // anchor -> norm/scale slot (0: circuit end)
    size_t next_slot_ = 1;
    mutable size_t ckpt_stride_ = 1;   // every stride-th boundary stores a checkpoint (max_ckpts >= 1)
    bool state_valid_ = false;
    bool have_result_ = false;

    // device scratch
    double *d_partials_ = nullptr;  size_t partials_cap_ = 0;
    double *d_scalars_ = nullptr;   size_t scalars_cap_ = 0;  // norms[slot], then scales[slot]
    unsigned long long *d_u64_ = nullptr;  size_t u64_cap_ = 0;
    uint64_t *d_mask_ = nullptr;    size_t mask_cap_ = 0;
    uint32_t *d_tiles_ = nullptr;   size_t tiles_cap_ = 0;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    bool dev_ready_ = false;
    bool tuned_ = false;

    // sizes the commit grows the scratch buffers to (0: unchanged)
    struct ScratchNeed {
        size_t scalars = 0, partials = 0, u64 = 0, tiles = 0, mask = 0;
    };
    ScratchNeed scratch_need() const;

    // prepared replay
    bool prep_pending_ = false;             // planned, not committed yet
    bool prep_committed_ = false;           // committed: the launch list is the current replay
    uint64_t prep_need_bytes_ = 0;
    std::vector<size_t> prep_list_off_;     // closed replay: tile-list offset per pass launch
    // sparse checkpoints: the state at the restart boundary put together
    // from the newest checkpoint holding each block (or |0...0>)
    struct RestorePart {
        uint64_t anchor = 0;               // source checkpoint (0: |0...0>)
        std::vector<uint32_t> dst, src;    // destination blocks, source blocks (buffer order)
    };
    std::vector<RestorePart> prep_restore_;
    uint32_t *d_restore_ = nullptr;
    size_t restore_cap_ = 0;               // uint32 entries
    size_t prep_s0_ = 0, prep_S_ = 0, prep_first_edit_ = 0;
    int prep_mode_ = 0;
    bool prep_renorm_ = false;
    BlockSet prep_set_;
    std::vector<uint32_t> prep_tiles_;
    double prep_t0_ = 0;
    friend struct SessionAccess;
};

}  // namespace qtask
