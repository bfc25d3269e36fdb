// Plan records shared by the host planner and the HIP pass kernel.
//
// A segment plan is one contiguous device blob laid out as
//   [KPass x n_pass][KStage x n_stage][KOp x n_op][coefficients (R) x n_coef]
// Offsets inside records are relative to the start of their own array.
//
// A pass works on tiles of 2^b amplitudes.  Tile bit p (0 <= p < b) stands
// for global qubit qlist[p]; qlist[0..c-1] = 0..c-1, so a tile is made of
// 2^(b-c) chunks of 2^c contiguous amplitudes.  The remaining n-b global
// bits enumerate the tiles.  Inside a workgroup the tile lives in LDS at a
// swizzled slot phys(l) (a GF(2)-linear map of the tile index l, so every
// offset below is an XOR of per-bit contributions).  A stage maps QK_G tile
// bits onto the QK_NREG registers of each thread and the other b-QK_G tile
// bits onto the thread index; its ops then run on registers.  Register i of
// a thread sits at the XOR (LDS slot) or OR (global offset) of the
// contributions of the set bits of i.
#pragma once
#include <stdint.h>

#define QK_G 4                // register bits per thread in a stage
#define QK_NREG 16            // 2^QK_G amplitudes per thread
#define QK_MAX_TILE_BITS 13
#define QK_MIN_TILE_BITS 4
#define QK_MAX_THR_BITS (QK_MAX_TILE_BITS - QK_G)
#define QK_MAX_QUBITS 34
#define QK_MAX_DENSE_K 6

enum KOpType : uint8_t {
    KOP_NONE = 0,
    KOP_U1 = 1,    // dense 2x2 on bit a                         coef: m00 m01 m10 m11 (8 reals)
    KOP_D1 = 2,    // diagonal on bit a                          coef: d0 d1 (4)
    KOP_A1 = 3,    // anti-diagonal on bit a                     coef: m01 m10 (4)
    KOP_X1 = 4,    // exact exchange on bit a                    coef: none
    // 5: unused
    KOP_CX = 6,    // exact exchange on bit b where bit a = 1    coef: none
    // 7: unused
    KOP_SWAP = 8,  // exact exchange of bits a and b             coef: none
    // 9: unused (two-qubit gates are exchanges or phases; stages with many
    //    ops become KOP_DENSE)
    KOP_CCX = 10,  // exact exchange on bit c where a = b = 1    coef: none
    KOP_DENSE = 11,// dense 16x16 on all QK_G register bits      coef: 512
    KOP_UR = 12,   // real 2x2 on bit a (H, RY)                 coef: m00 m01 m10 m11 (4 reals)
    KOP_UX = 13,   // [[a, ib], [ic, d]] with a,b,c,d real (RX)  coef: a b c d (4)
    KOP_P1 = 14,   // diag(1, p) on bit a (Z, S, T, ...)         coef: p (2)
    KOP_P2 = 15,   // diag(1, 1, 1, p) on (a, b) (CZ, CP)        coef: p (2)
    KOP_GPH = 16,  // every amplitude times g (no qubits)       coef: g (2)
    KOP_PC = 17,   // phase p on the registers with bit a set, in the lanes where site b
                   // (a lane or origin site code, below) is 1      coef: p (2)
    KOP_PCL = 18,  // phase p for every register of the lanes where sites a and b are 1:
                   // multiplied into the lane's pending factor    coef: p (2)
    KOP_PHI = 19   // every register times the lane's pending factor (where one was
                   // taken), which then resets to 1             coef: none
};

// Site codes of the phase ops: where a phase gate's qubit sits in the stage.
#define KPC_LANE 16      // 16 + k: bit k of the thread index
#define KPC_ORIGIN 64    // 64 + q: bit q of the tile's global origin (the qubit is not in the tile)
#define KPC_NONE 255     // no qubit (the condition always holds)

enum KStageKind : uint32_t {
    KSTAGE_LIST = 0,   // ops on registers (vector ALU)
    KSTAGE_MFMA = 1    // one dense 2^k x 2^k unitary on the matrix cores
};

struct KOp {
    uint8_t type, a, b, c;  // register bit positions (a = first-listed qubit = high local bit)
    uint32_t coef;          // offset into the coefficient array (in R units)
};

// The first 64 bytes of a stage (register and thread maps, op range, kind)
// are what every stage of every tile needs; the kernel reads them with one
// scalar load.
struct KStage {
    uint32_t reg_bit[QK_G];           // LDS slot contribution of register-index bit j
    uint32_t thr_off[QK_MAX_THR_BITS];// LDS slot contribution of thread-index bit k
    uint32_t op_begin, op_count;      // ops of the stage; consecutive stages have consecutive ranges
    uint32_t kind;                    // KStageKind
    uint64_t g_bit[QK_G];             // first/last stage: global offset of register-index bit j
    uint64_t g_thr[QK_MAX_THR_BITS];  // first/last stage: global offset of thread-index bit k
    uint32_t k;                       // MFMA stage: qubits of the dense unitary
    uint32_t coef;                    // MFMA stage: offset of the real block operand in lane order (16-value aligned)
    uint32_t n_col_bits;              // MFMA stage: b - k
    uint32_t row_off[1 << QK_MAX_DENSE_K]; // MFMA stage: LDS slot of row r (the k stage bits)
    uint32_t col_off[QK_MAX_TILE_BITS];    // MFMA stage: LDS slot contribution of column bit
};

// A pass: its first stage loads its registers straight from global memory and
// its last stage stores straight from registers (both through their own
// global maps, chosen so that consecutive lanes touch consecutive
// addresses); the stages in between exchange data through LDS.
// The global offset of a tile is its index with bits deposited at the
// non-tile qubits.  Those qubits form at most b + 1 runs of consecutive
// positions; run r moves tile-index bits [src, src + len) to global bits
// [dst, dst + len), packed as src | len << 8 | dst << 16.
#define QK_MAX_RUNS (QK_MAX_TILE_BITS + 1)

struct KPass {
    uint8_t nonq_pos[QK_MAX_QUBITS];    // global bit of tile-index bit k
    uint8_t pad[2];
    uint32_t n_nonq;                    // n - b
    uint32_t n_thr;                     // b - QK_G
    uint32_t stage_begin, stage_count;  // stage_count >= 1
    uint32_t n_runs;                    // runs of consecutive non-tile qubits
    uint32_t run[QK_MAX_RUNS];          // deposit runs (see above)
};

// Launch arguments of one pass (passed by value).
struct KArgs {
    void *dst;                 // state written by the pass
    const void *src;           // state read by the pass (may equal dst)
    void *ckpt;                // optional second destination (checkpoint), or null
    const KPass *pass;
    const KStage *stages;
    const KOp *ops;
    const void *coefs;         // R array
    const uint32_t *tile_list; // optional: blockIdx -> tile index
    const uint64_t *store_mask;// optional: store only blocks whose bit is set
    const double *scale;       // optional: multiply loaded amplitudes by (R)*scale
    double *partials;          // optional: per-tile sum |a|^2 in FP64 (indexed by blockIdx)
    uint32_t src_basis;        // 1: the input is |0...0> (src unused)
    uint32_t block_bits;       // store_mask granularity
    uint32_t has_mfma;         // the pass has matrix-core stages
    uint32_t has_dense;        // the pass has dense 16x16 register ops (KOP_DENSE)
};

// Work item of the batched small-session launch.
struct KBatchItem {
    KArgs args;
    uint32_t tile_begin;       // first global workgroup index of this item
    uint32_t n_tiles;
    uint32_t threads;          // 2^(b - QK_G) threads used by this item
    uint32_t pad;
};

// Renormalisation sum of one batched item.
struct KSumItem {
    const double *partials;
    double *norm_out;
    double *scale_out;
    uint32_t n;
    uint32_t pad;
};
