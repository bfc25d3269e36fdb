/*
 * qtask.h -- C ABI of the MI355X incremental state-vector library (libqtask.so).
 *
 * The programming model follows the qTask paper (Section III-B, Table II and
 * Listing 1): a circuit of n qubits is an ordered list of nets ("levels"),
 * each net a set of gates on disjoint qubits.  Three groups of calls exist:
 * circuit modifiers (insert/remove a level or a gate), the state update
 * (first call simulates the whole circuit, later calls re-simulate only what
 * the modifiers since the previous update affect, Section III-E), and
 * queries (amplitudes, norm, inner product, statistics, plan dump).
 *
 * Conventions
 *  - Qubit k is bit k of the amplitude index (the last qubit is the most
 *    significant bit, Section III-B).  The state starts as |0...0>.
 *  - Gate qubits are listed controls first, then target(s).  For a k-qubit
 *    gate on (q0, ..., q_{k-1}) the local index of its matrix is
 *    bit(q0)*2^(k-1) + ... + bit(q_{k-1}), i.e. the first-listed qubit is the
 *    high bit (the CX matrix of Section II-A has its control on the high bit).
 *  - Rotations are RX/RY/RZ(theta) = exp(-i theta P/2); S = diag(1,i) and
 *    T = diag(1,e^{i pi/4}) (Table I); CP(lambda) = diag(1,1,1,e^{i lambda}).
 *  - Amplitudes are interleaved (re, im) pairs: double for QTASK_C128, float
 *    for QTASK_C64.
 *
 * Status and errors
 *  Every call returns an int status (QTASK_OK or a QTASK_E_* code).  No C++
 *  exception crosses the ABI.  A call that fails leaves the circuit, the state
 *  and every output argument unchanged (strong guarantee), except that
 *  QTASK_E_DEVICE from qtask_update_state leaves the state undefined until the
 *  next successful update (the circuit is unchanged and the next update
 *  re-simulates from scratch).
 *
 * Ownership and threading
 *  Handles are owned by the caller until the matching destroy call.  Device
 *  memory (state and checkpoints) is owned by the library and allocated
 *  through the allocator hooks of qtask_opts (hipMalloc when NULL).  Host
 *  buffers passed in are caller-owned and never retained.  A handle must not
 *  be used by two threads at once; distinct handles are independent.  Level
 *  and gate ids stay valid until the level/gate is removed; ids are never
 *  reused within a handle.
 */
#ifndef QTASK_API_H_
#define QTASK_API_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define QTASK_OK            0
#define QTASK_E_ARG         1  /* bad argument: qubit out of range, repeated qubit, wrong parameter count, NULL pointer */
#define QTASK_E_CONFLICT    2  /* the gate shares a qubit with a gate already in that level (paper: insert into a net that introduces a dependency is rejected, Section III-B) */
#define QTASK_E_NOTFOUND    3  /* stale or unknown level/gate id, or index out of range */
#define QTASK_E_NOMEM       4  /* device allocation failed, or a serving budget cannot admit the session */
#define QTASK_E_DEVICE      5  /* a HIP call failed */
#define QTASK_E_STALE       6  /* state queried while modifiers are pending since the last update */
#define QTASK_E_UNSUPPORTED 7  /* valid request that the library or this session mode does not support */
#define QTASK_E_BUSY        8  /* the handle is owned by a server and has work in flight */

typedef enum qtask_dtype {
    QTASK_C128 = 0, /* complex128 amplitudes, FP64 arithmetic */
    QTASK_C64 = 1   /* complex64 amplitudes, FP32 arithmetic, FP64 reductions */
} qtask_dtype;

typedef enum qtask_gate_kind {
    QTASK_H = 0, QTASK_X, QTASK_Y, QTASK_Z, QTASK_S, QTASK_SDG, QTASK_T, QTASK_TDG,
    QTASK_RX, QTASK_RY, QTASK_RZ,          /* one angle parameter */
    QTASK_CX, QTASK_CZ, QTASK_SWAP,
    QTASK_CP,                              /* one angle parameter */
    QTASK_CCX,                             /* Toffoli: controls first */
    QTASK_GATE_KIND_COUNT
} qtask_gate_kind;

typedef enum qtask_fusion {
    QTASK_FUSE_AUTO = 0,  /* per stage: gate list on the vector ALU, or one dense
                             unitary on the matrix cores when that is cheaper */
    QTASK_FUSE_NONE = 1,  /* gate lists only */
    QTASK_FUSE_DENSE = 2  /* every stage becomes one dense fuse_width-qubit unitary */
} qtask_fusion;

#define QTASK_DEVICE_NONE (-1) /* plan-only session: circuit store, planner and
                                  tracker run, nothing is allocated or launched,
                                  amplitude queries return QTASK_E_UNSUPPORTED */
#define QTASK_FRONT ((uint64_t)0) /* "insert before the first level" */

/* Options for qtask_create.  Zero-initialise, set struct_size, then override
 * fields (or call qtask_opts_default).  0 in a tuning field means "choose". */
typedef struct qtask_opts {
    uint32_t struct_size;   /* sizeof(qtask_opts) */
    int32_t device;         /* HIP device ordinal, or QTASK_DEVICE_NONE */
    int32_t tile_bits;      /* b: a pass works on tiles of 2^b amplitudes (4..13) */
    int32_t low_bits;       /* c: every tile holds 2^c contiguous amplitudes (c <= b) */
    int32_t block_bits;     /* tracker block = 2^block_bits contiguous amplitudes (the paper's block size B = 2^block_bits, Section III-C) */
    int32_t fusion;         /* qtask_fusion */
    int32_t fuse_width;     /* k for QTASK_FUSE_DENSE (2..6) */
    int32_t ckpt_interval;  /* levels per checkpoint segment (default 100) */
    int32_t max_ckpts;      /* at most this many device checkpoints; -1 = unlimited */
    int32_t renorm;         /* C64: renormalise at every segment end (default 1) */
    int32_t autotune;       /* 1: time candidate (tile_bits, low_bits) at the first update and keep the fastest
                               (every candidate on a prefix of about 600 gates, the three fastest again on the
                               first segments, about 3000 gates; within 1% the smaller tile wins); under QTASK_FUSE_AUTO the
                               candidates also include dense fusion at fuse_width 4..6, and the pick sets fusion
                               and fuse_width.  The pick is cached per process and frozen for the session */
    int32_t closed_mode;    /* 1 (default): replay only affected blocks when the affected set is closed */
    void *stream;           /* hipStream_t for all work; NULL = a library-owned stream */
    void *(*alloc)(size_t bytes, void *ctx); /* device allocator; NULL = hipMalloc.  Must return memory aligned to
                                                 256 bytes (as hipMalloc does); other memory is freed and the
                                                 allocation fails */
    void (*free)(void *ptr, void *ctx);
    void *alloc_ctx;
    int32_t relabel;        /* qubit relabelling inside checkpoint segments: 1 on, 0 off, -1 (default) on for
                               states of 26 or more qubits.  A pass may store its tile with the qubits
                               permuted among the tile's positions, so that the qubits the next passes need
                               sit in the contiguous low positions every tile holds (longer contiguous runs
                               per access at the same number of passes); each segment starts and ends in
                               the plain layout (qubit k at bit k), so checkpoints and queries see it */
    int32_t ckpt_delta;     /* 1: sparse checkpoints (the paper's copy-on-write blocks, Section III-F): a
                               stored boundary's checkpoint holds only the blocks of 2^block_bits amplitudes that
                               the segments since the previous stored boundary can change (decided by the ops'
                               kernel forms); a restore takes each block from the newest stored checkpoint holding
                               it, |0...0> where none does.  max_ckpts thins the stored boundaries as for whole
                               copies.  The affected-block replay (mode 3) is not used with them.  0 (default):
                               whole copies */
} qtask_opts;

typedef struct qtask_s *qtask_t;
typedef uint64_t qtask_level_t;
typedef uint64_t qtask_gate_t;

typedef struct qtask_stats {
    uint32_t struct_size;
    int32_t mode;              /* 0 nothing to do, 1 full, 2 incremental (whole state), 3 incremental (affected blocks only) */
    uint64_t levels_total;
    uint64_t levels_replayed;
    uint64_t segments_replayed;
    uint64_t first_level;      /* first level index re-simulated */
    uint64_t passes;           /* pass kernels launched (passes with no tile to run are skipped) */
    uint64_t tiles;            /* tiles processed over all passes */
    uint64_t stages;           /* stages over all passes (per tile) */
    uint64_t dirty_blocks;     /* blocks in the affected set (mode 3), else all blocks */
    uint64_t total_blocks;
    uint64_t gate_amp_updates; /* sum over replayed gates of 2^n */
    double bytes;              /* algorithmic HBM bytes of the launched kernels */
    double flops;              /* algorithmic flops of the launched kernels */
    double mfma_flops;         /* the part of `flops` done by dense fused unitaries on the matrix cores */
    double kernel_ms;          /* device time from the first to the last launched kernel */
    double pass_kernel_ms;     /* device time of the pass kernels alone */
    double plan_ms;            /* host planning time */
    double wall_ms;            /* wall time of the call */
    uint64_t ckpt_bytes;       /* device bytes the stored checkpoints hold after the call */
    uint64_t ckpt_full_bytes;  /* the same checkpoints as whole-state copies */
} qtask_stats;

/* ---------------------------------------------------------------- basics */
const char *qtask_status_string(int status);
int qtask_version(int *major, int *minor);
/* Text of the last error recorded on the handle ("" if none); valid until the
 * next call on the handle. */
const char *qtask_last_error(qtask_t h);
int qtask_opts_default(qtask_opts *opts);
/* Number of HIP devices visible (0 when none); never fails. */
int qtask_device_count(int *count);

/* Create a circuit of n_qubits (1..34) qubits with no levels.  opts may be
 * NULL (defaults).  Device memory is allocated at the first update. */
int qtask_create(int n_qubits, qtask_dtype dtype, const qtask_opts *opts, qtask_t *out);
int qtask_destroy(qtask_t h);

/* ------------------------------------------------------ circuit modifiers */
/* Insert an empty level right after level `after` (QTASK_FRONT: before the
 * first level).  Paper: insert_net (Table II). */
int qtask_insert_level(qtask_t h, qtask_level_t after, qtask_level_t *out);
/* Remove a level and all its gates.  Paper: remove_net (Table II). */
int qtask_remove_level(qtask_t h, qtask_level_t level);
/* Insert a gate into a level.  qubits: nq qubits, controls first; params: np
 * angles (RX/RY/RZ/CP take 1, others 0).  QTASK_E_CONFLICT when a qubit is
 * already used in that level.  Paper: insert_gate (Table II). */
int qtask_insert_gate(qtask_t h, qtask_level_t level, qtask_gate_kind kind,
                      const int32_t *qubits, int nq, const double *params, int np,
                      qtask_gate_t *out);
/* Remove a gate from its level.  Paper: remove_gate (Table II). */
int qtask_remove_gate(qtask_t h, qtask_gate_t gate);
int qtask_num_levels(qtask_t h, uint64_t *out);
int qtask_level_at(qtask_t h, uint64_t index, qtask_level_t *out);
int qtask_num_gates(qtask_t h, uint64_t *out);

/* ----------------------------------------------------------- state update */
/* Bring the state up to date with the circuit.  The first call simulates
 * everything; later calls restore the newest valid checkpoint at or before
 * the first modified level and re-simulate from there, touching only the
 * affected blocks when that set is closed (Section III-E).  Blocking.  The
 * result is bitwise identical to qtask_update_state_full on the same
 * circuit and options.
 * Errors: the update first plans on the host, then allocates every device
 * buffer it needs (plans, state, new checkpoints, scratch; through the
 * allocator hooks of qtask_opts when set) before it changes any of them.
 * QTASK_E_NOMEM (an allocation failed) and QTASK_E_ARG (a plan could not be
 * built) therefore leave the previous result, its checkpoints and their
 * validity as they were; the modifiers stay pending, so amplitude queries
 * return QTASK_E_STALE until an update succeeds, and that update resumes
 * from the same checkpoints.  QTASK_E_DEVICE leaves the state undefined and
 * the next update re-simulates from |0...0>. */
int qtask_update_state(qtask_t h);
/* Re-simulate the whole circuit from |0...0>, ignoring checkpoints. */
int qtask_update_state_full(qtask_t h);
/* Statistics of the last update call. */
int qtask_last_update_stats(qtask_t h, qtask_stats *out);

/* ------------------------------------------------------------------ query */
/* Copy amplitudes [first, first+count) to host_out (interleaved re,im in the
 * session dtype).  QTASK_E_STALE if modifiers are pending, QTASK_E_NOTFOUND
 * if the range exceeds 2^n. */
int qtask_read_amplitudes(qtask_t h, uint64_t first, uint64_t count, void *host_out);
/* sum_b |alpha_b|^2 accumulated in FP64 with a fixed reduction order. */
int qtask_norm(qtask_t h, double *out);
/* <a|b> accumulated in FP64 (re, im); a and b must have the same n and
 * device; their dtypes may differ (a complex64 state against its complex128
 * reference). */
int qtask_inner(qtask_t a, qtask_t b, double re_im[2]);
/* qtask_inner without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The partial sums go to a fixed scratch array the
 * library holds on each GPU until the process ends (4098 doubles, 32 KiB:
 * enough for the reduction of any state up to 34 qubits, so no state size
 * is refused; QTASK_E_UNSUPPORTED would name one that is).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (from several
 * threads, or on several streams) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero: each call writes
 * every partial it reads.  Same arguments, layout and errors as
 * qtask_inner. */
int qtask_inner_noalloc(qtask_t a, qtask_t b, double re_im[2]);
/* Number of amplitude slots whose bytes differ between a and b (bitwise). */
int qtask_compare_states(qtask_t a, qtask_t b, uint64_t *n_diff);
/* Deterministic 64-bit hash of the state bytes. */
int qtask_state_hash(qtask_t h, uint64_t *out);
/* Device pointer and size in bytes of the current state (read-only use;
 * valid until the next update or destroy). */
int qtask_state_device_ptr(qtask_t h, const void **ptr, uint64_t *bytes);
/* Device bytes held by the session (state, checkpoints, plans and scratch). */
int qtask_device_bytes(qtask_t h, uint64_t *out);
/* The options in effect (after defaults and autotuning). */
int qtask_get_opts(qtask_t h, qtask_opts *out);
/* Write the current plan (passes, stages, ops, fused unitaries, affected
 * blocks of the last update) as JSON to `path`.  A path ending in ".dot"
 * gets the pass graph in Graphviz DOT instead: one cluster per segment, one
 * node per pass in execution order, checkpoint boundaries marked.  Paper:
 * dump_graph (Table II).  QTASK_E_ARG if the file cannot be written. */
int qtask_dump_plan(qtask_t h, const char *path);

/* ----------------------------------------------------------- diagnostics */
/* Bandwidth of a plain device copy kernel: copies `bytes` (rounded down to
 * 256 B) between two fresh device buffers `iters` times and returns the
 * achieved (read + write) GB/s.  This is the measured ceiling the pass
 * kernels are compared against. */
int qtask_copy_bandwidth(int device, uint64_t bytes, int iters, double *gbps);

/* --------------------------------------------------------------- serving */
/* A server keeps many sessions resident on one device and runs their update
 * requests with continuous batching: requests that arrive while others run
 * are started as soon as device memory and a launch slot free up, sessions
 * above the small-session threshold run on their own streams, and sessions
 * below it are packed into one batched launch per pass round replayed from a
 * captured HIP graph. */
typedef struct qtask_server_s *qtask_server_t;

typedef struct qtask_server_opts {
    uint32_t struct_size;
    int32_t device;
    uint64_t budget_bytes;    /* device bytes the sessions may hold together: state, checkpoints, plans and
                                 per-session scratch (the server's own tables and the transient buffers of
                                 a first-update autotune are not charged) */
    int32_t max_inflight;     /* large sessions updating at once */
    int32_t small_qubits;     /* sessions with n < small_qubits go through the batched graph launch (default 16) */
    int32_t use_graph;        /* 1 (default): capture the batched launch in a HIP graph */
    int32_t order;            /* which waiting request starts first: 0 (default) the oldest; 1 the one whose
                                 update is expected to be shortest (2^n times the session's levels), that
                                 estimate divided by 1 + waiting time / 1 s so that no request waits for ever */
} qtask_server_opts;

typedef struct qtask_edit {
    int32_t op;               /* 0 insert gate, 1 remove gate, 2 insert level, 3 remove level */
    int32_t kind;             /* qtask_gate_kind (insert gate) */
    uint64_t level;           /* level index (insert gate / remove level) or index after which to insert (insert level; UINT64_MAX = front) */
    uint64_t gate_index;      /* remove gate: index of the gate within the level, in insertion order */
    int32_t qubits[3];
    int32_t nq;
    double params[3];
    int32_t np;
} qtask_edit;

typedef struct qtask_result {
    uint64_t ticket;
    int32_t status;
    int32_t session;
    double submit_ms;         /* server clock when submitted */
    double start_ms;          /* when its update started on the device */
    double done_ms;           /* when its update finished */
    double latency_ms;        /* done - submit */
    uint64_t state_hash;      /* qtask_state_hash of the session after the update */
    qtask_stats stats;
} qtask_result;

int qtask_server_opts_default(qtask_server_opts *opts);
int qtask_server_create(const qtask_server_opts *opts, qtask_server_t *out);
/* Waits for all work, then frees every session it owns. */
int qtask_server_destroy(qtask_server_t s);
/* Open a session of n qubits with the given nets already built: gates are
 * given as flat arrays (kinds, qubits 3 per gate, params 3 per gate, nq per
 * gate) with level_of_gate[i] the level index of gate i; n_levels levels are
 * created.  Memory is charged when the session is admitted (its first
 * request), not here.  Returns the session index. */
int qtask_server_open(qtask_server_t s, int n_qubits, qtask_dtype dtype, const qtask_opts *opts,
                      uint64_t n_levels, uint64_t n_gates, const int32_t *kinds,
                      const int32_t *qubits, const int32_t *nq, const double *params,
                      const uint64_t *level_of_gate, int32_t *session_out);
/* Queue a request: apply the edits, then update the state.  Returns at once.
 * A request is admitted by the bytes its session holds after the update
 * (edits that add levels can add checkpoints), evicting idle sessions
 * least recently used first; it waits while that does not fit.  A request
 * is all or nothing: when an edit fails, or the update fails with anything
 * but QTASK_E_DEVICE (including QTASK_E_NOMEM for a session that can never
 * fit the budget), its edits are undone and the session keeps its previous
 * state. */
int qtask_server_submit(qtask_server_t s, int32_t session, const qtask_edit *edits, int n_edits,
                        uint64_t *ticket_out);
/* Block until the ticket's request finished (timeout_ms < 0: no limit). */
int qtask_server_wait(qtask_server_t s, uint64_t ticket, double timeout_ms, qtask_result *out);
/* Non-blocking: 1 in *done when finished (and *out filled), else 0. */
int qtask_server_poll(qtask_server_t s, uint64_t ticket, int *done, qtask_result *out);
/* Block until every submitted request finished. */
int qtask_server_drain(qtask_server_t s);
/* Borrow the session handle for queries (only while it has no work queued;
 * QTASK_E_BUSY otherwise). */
int qtask_server_session(qtask_server_t s, int32_t session, qtask_t *out);
/* Device bytes currently admitted, and sessions resident. */
int qtask_server_usage(qtask_server_t s, uint64_t *bytes, int32_t *resident);
/* Largest value the admitted bytes reached since the server was created
 * (never above budget_bytes). */
int qtask_server_peak_bytes(qtask_server_t s, uint64_t *peak);
/* Where the server's requests ran, since it was created: *batched counts
 * requests started in batched ticks (small sessions, any pass kernel
 * variant), *streamed requests launched on their session's own stream
 * (large sessions, and plans with sparse-checkpoint block copies), *ticks
 * the batched ticks. */
int qtask_server_paths(qtask_server_t s, uint64_t *batched, uint64_t *streamed, uint64_t *ticks);

#ifdef __cplusplus
}
#endif
#endif /* QTASK_API_H_ */
