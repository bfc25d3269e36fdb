// Affected-block tracker.
//
// The paper restarts an update from "frontier" partitions (the partitions of
// inserted gates and the successors of removed ones) and re-runs every
// partition reachable from them (Section III-E).  Here the state is cut into
// blocks of 2^beta contiguous amplitudes (the paper's block size B = 2^beta,
// Section III-C) and the same reachability is computed directly on block
// sets: a gate's touched blocks are the blocks holding an amplitude the gate
// can change, and a gate that moves amplitude between blocks (a non-diagonal
// action on a qubit >= beta) spreads "affected" from a block to the blocks it
// couples with.
#pragma once
#include <cstdint>
#include <functional>
#include <vector>

#include "lowering.h"

namespace qtask {

class BlockSet {
public:
    BlockSet() = default;
    BlockSet(uint64_t nblocks, bool full = false) { reset(nblocks, full); }
    void reset(uint64_t nblocks, bool full);
    uint64_t size() const { return n_; }
    bool test(uint64_t j) const { return (w_[j >> 6] >> (j & 63)) & 1; }
    void set(uint64_t j) { w_[j >> 6] |= uint64_t(1) << (j & 63); }
    uint64_t count() const;
    bool all() const { return count() == n_; }
    void merge(const BlockSet &o);
    const std::vector<uint64_t> &words() const { return w_; }
    std::vector<uint32_t> list() const;

private:
    uint64_t n_ = 0;
    std::vector<uint64_t> w_;
};

// Which blocks an op reads from which, as the kernel runs it.  The coupling
// follows the op's kernel form, not its matrix values: a dense 2x2 (or a fused
// dense stage) reads every amplitude of its group even where its matrix has
// an exact zero, and the product 0 * x still decides the sign of a zero
// result, so a block it pairs with a stale partner could come out with
// different bits.  Diagonal ops read nothing across blocks; exchanges read
// exactly the partner they move.
struct BlockAction {
    uint64_t hmask = 0;            // block-index bits of the gate's qubits >= beta
    int nh = 0;                    // number of such qubits (at most QK_MAX_DENSE_K)
    std::vector<uint8_t> couple;   // couple[h_out * 2^nh + h_in]: h_out != h_in mix
    bool any_couple = false;
    std::vector<int> hq;           // block-index bit of high qubit i (i-th in hmask order)
};

BlockAction block_action(const LGate &g, int beta);

// A fused dense stage on the given qubits: every amplitude of a group reads
// every other one.
BlockAction dense_action(const std::vector<int> &qubits, int beta);

// Blocks whose amplitudes the kernel rewrites when it runs this op (decided
// by the op's kernel form, not by matrix values): controlled and phase ops
// rewrite only the amplitudes with their control/phase bits set, every other
// op rewrites its whole support.  Calls f(block) for each such block.
void for_rewritten_blocks(const LGate &g, int beta, uint64_t nblocks, const std::function<void(uint64_t)> &f);
// True when for_rewritten_blocks would visit every block (no control or
// phase bit at or above beta restricts the op).
bool rewrites_every_block(const LGate &g, int beta);

// d |= blocks coupled to d by the gate
void propagate(const BlockAction &a, BlockSet &d);
// true when the gate couples no block of s with a block outside s
bool closed_under(const BlockAction &a, const BlockSet &s);

}  // namespace qtask
