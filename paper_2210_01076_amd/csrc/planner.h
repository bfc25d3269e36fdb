// Planner: turns the ops of one checkpoint segment into passes over the
// state (each pass = one read and one write of every tile) and, inside a
// pass, into stages of register-resident work.
#pragma once
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "kdefs.h"
#include "lowering.h"

namespace qtask {

struct PlanParams {
    int n = 0;          // qubits of the state buffer (>= QK_MIN_TILE_BITS)
    int b = 12;         // tile bits
    int c = 4;          // contiguous low bits per tile
    int dtype = 0;      // 0 complex128, 1 complex64
    int fusion = 0;     // qtask_fusion
    int fuse_k = 4;     // width of dense fused unitaries
    int swz = 4;        // LDS swizzle width in bits
    int relabel = 0;    // 1: passes may relabel qubits (see PPass::out)
};

struct PStage {
    std::vector<int> tbits;   // tile bits of the stage's register index bits (ascending)
    std::vector<int> tpos;    // tile bits of the thread index (lane-friendly order)
    std::vector<LGate> ops;   // ops in program order (global qubits)
    bool mfma = false;        // one dense unitary on the matrix cores
    std::vector<cd> U;        // fused unitary, register-index convention (MFMA and KOP_DENSE)
    double flops = 0;         // algorithmic flops per amplitude
};

// Qubit relabelling.  Ops and tile bits name physical bit positions of the
// state buffer.  Without relabelling a circuit qubit always sits at its own
// position; with it, a pass may store tile bit p at position out[p] instead
// of qlist[p] (a permutation of the tile's positions), so that the qubits
// the next passes need come to sit in the contiguous low positions every
// tile holds.  Each segment starts and ends with every qubit at its own
// position, so checkpoints and the final state keep the plain layout.
struct PPass {
    std::vector<int> qlist;   // physical position of tile bit p (where it is loaded from)
    std::vector<int> out;     // physical position tile bit p is stored to (empty: qlist)
    std::vector<PStage> stages;
    uint64_t qmask = 0;
    int n_gates = 0;          // source gates applied in this pass
    bool has_mfma = false;    // some stage runs on the matrix cores
    bool has_dense = false;   // some stage is a dense 16x16 op on registers
    bool relabels() const { return !out.empty() && out != qlist; }
    int out_pos(int p) const { return out.empty() ? qlist[size_t(p)] : out[size_t(p)]; }
};

// A phase the kernel folds into each lane's pending factor: the global phase,
// or a phase gate none of whose qubits is on the stage's registers.  Such ops
// run after the stage's other ops, multiplied together first, and the
// product then scales the lane's registers once.
bool lane_phase(const PPass &ps, const PStage &st, const LGate &g);

struct SegmentPlan {
    PlanParams pp;
    std::vector<PPass> passes;
    std::vector<uint8_t> blob;         // packed KPass | KStage | KOp | coefficients
    size_t off_stage = 0, off_op = 0, off_coef = 0;
    uint64_t n_gates = 0;
    double flops_per_amp = 0;          // summed over passes
    uint64_t hash = 0;                 // content + parameters
    void *dev = nullptr;               // device copy of blob
    size_t dev_bytes = 0;
};

// Plan a segment.  `ops` are the lowered gates of the segment's levels in
// canonical order (level by level; inside a level by lowest qubit).  `hash`
// is segment_hash(ops, pp) when the caller has it (0: computed here).
SegmentPlan plan_segment(const std::vector<LGate> &ops, const PlanParams &pp, uint64_t hash = 0);

// Hash of a segment's content and the parameters that shape its plan.
uint64_t segment_hash(const std::vector<LGate> &ops, const PlanParams &pp);

// One 64-bit word into a running hash, through a splitmix finalizer.  Every
// bit of the word reaches every bit of the result (an xor-multiply step
// would not do: flipping the top bit of two words, as negating a complex
// number does, cancels out in it).
inline uint64_t hash_mix(uint64_t h, uint64_t w) {
    uint64_t x = h + w * 0x9e3779b97f4a7c15ull;
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Bit pattern of a double, for hashing.
inline uint64_t double_bits(double v) {
    uint64_t b;
    std::memcpy(&b, &v, sizeof(b));
    return b;
}

// LDS slot of tile index l under the swizzle of width `swz`.
uint32_t lds_phys(uint32_t l, int swz);

// Check that every table of the plan is a bijection onto the tile and that
// every op sits inside its stage and pass; returns "" or a description.
std::string validate_plan(const SegmentPlan &sp);

// JSON description of a plan (passes, stages, ops, fused unitaries).
std::string plan_json(const SegmentPlan &sp, bool with_matrices);

}  // namespace qtask
