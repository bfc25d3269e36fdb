#include "tracker.h"

#include <algorithm>
#include <stdexcept>

namespace qtask {

void BlockSet::reset(uint64_t nblocks, bool full) {
    n_ = nblocks;
    w_.assign((nblocks + 63) / 64, full ? ~uint64_t(0) : 0);
    if (full && (nblocks & 63)) w_.back() = (uint64_t(1) << (nblocks & 63)) - 1;
}

uint64_t BlockSet::count() const {
    uint64_t c = 0;
    for (uint64_t x : w_) c += uint64_t(__builtin_popcountll(x));
    return c;
}

void BlockSet::merge(const BlockSet &o) {
    for (size_t i = 0; i < w_.size(); ++i) w_[i] |= o.w_[i];
}

std::vector<uint32_t> BlockSet::list() const {
    std::vector<uint32_t> out;
    for (size_t i = 0; i < w_.size(); ++i) {
        uint64_t x = w_[i];
        while (x) {
            const int b = __builtin_ctzll(x);
            out.push_back(uint32_t(i * 64 + b));
            x &= x - 1;
        }
    }
    return out;
}

namespace {

// Block structure of an op on the given qubits whose kernel reads entry
// (r, c) of its matrix where reads(r, c) holds (local bit of qubit j is
// k-1-j).
template <typename Reads>
BlockAction make_action(const int *q, int k, int beta, Reads &&reads) {
    BlockAction a;
    const int dim = 1 << k;
    // split the local index into its high part (qubits >= beta, ascending
    // by qubit) and the rest
    std::vector<int> hi_j;  // gate qubit indices j with q >= beta
    for (int j = 0; j < k; ++j)
        if (q[j] >= beta) hi_j.push_back(j);
    std::sort(hi_j.begin(), hi_j.end(), [&](int x, int y) { return q[x] < q[y]; });
    a.nh = int(hi_j.size());
    if (a.nh > QK_MAX_DENSE_K) throw std::logic_error("op on too many block qubits");
    for (int j : hi_j) {
        a.hmask |= uint64_t(1) << (q[j] - beta);
        a.hq.push_back(q[j] - beta);
    }
    const int hd = 1 << a.nh;
    auto hpart = [&](int local) {
        int h = 0;
        for (int i = 0; i < a.nh; ++i) h |= ((local >> (k - 1 - hi_j[i])) & 1) << i;
        return h;
    };
    a.couple.assign(size_t(hd) * hd, 0);
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            if (hpart(r) != hpart(c) && reads(r, c)) {
                a.couple[size_t(hpart(r)) * hd + hpart(c)] = 1;
                a.any_couple = true;
            }
    return a;
}

}  // namespace

BlockAction block_action(const LGate &g, int beta) {
    const int k = g.nq, dim = 1 << k;
    switch (g.kop) {
    case KOP_D1: case KOP_P1: case KOP_P2: case KOP_GPH:
        return make_action(g.q, k, beta, [](int, int) { return false; });
    case KOP_X1: case KOP_CX: case KOP_SWAP: case KOP_CCX:
        // exact exchanges: the matrix is the permutation the kernel moves by
        return make_action(g.q, k, beta, [&](int r, int c) { return g.m[size_t(r) * dim + c] != cd(0, 0); });
    default:  // dense forms: every entry of a row is read
        return make_action(g.q, k, beta, [](int, int) { return true; });
    }
}

BlockAction dense_action(const std::vector<int> &qubits, int beta) {
    return make_action(qubits.data(), int(qubits.size()), beta, [](int, int) { return true; });
}

void for_rewritten_blocks(const LGate &g, int beta, uint64_t nblocks, const std::function<void(uint64_t)> &f) {
    // required-one bits (as block-index bits) and, for SWAP, a pair that must differ
    uint64_t need = 0;
    bool all = false, swap_hi = false;
    int sa = -1, sb = -1;
    auto hb = [&](int q) { return q >= beta ? int(q - beta) : -1; };
    switch (g.kop) {
    case KOP_P1:
        if (hb(g.q[0]) >= 0) need |= uint64_t(1) << hb(g.q[0]);
        break;
    case KOP_P2:
        for (int j = 0; j < 2; ++j)
            if (hb(g.q[j]) >= 0) need |= uint64_t(1) << hb(g.q[j]);
        break;
    case KOP_CX:
        if (hb(g.q[0]) >= 0) need |= uint64_t(1) << hb(g.q[0]);
        break;
    case KOP_CCX:
        for (int j = 0; j < 2; ++j)
            if (hb(g.q[j]) >= 0) need |= uint64_t(1) << hb(g.q[j]);
        break;
    case KOP_SWAP:
        sa = hb(g.q[0]);
        sb = hb(g.q[1]);
        swap_hi = sa >= 0 && sb >= 0;
        break;
    default:
        all = true;
        break;
    }
    for (uint64_t j = 0; j < nblocks; ++j) {
        if (all) { f(j); continue; }
        if ((j & need) != need) continue;
        if (swap_hi && (((j >> sa) & 1) == ((j >> sb) & 1))) continue;
        f(j);
    }
}

bool rewrites_every_block(const LGate &g, int beta) {
    switch (g.kop) {
    case KOP_P1: case KOP_CX: return g.q[0] < beta;
    case KOP_P2: case KOP_CCX: return g.q[0] < beta && g.q[1] < beta;
    case KOP_SWAP: return !(g.q[0] >= beta && g.q[1] >= beta);
    default: return true;
    }
}

namespace {
// Visit every group of 2^nh blocks that differ only in the gate's high bits:
// f(blocks[2^nh]) with blocks[h] the block index whose high part is h.
template <typename F>
void for_groups(const BlockAction &a, uint64_t nblocks, F &&f) {
    const int hd = 1 << a.nh;
    uint64_t idx[1 << QK_MAX_DENSE_K];
    for (uint64_t base = 0; base < nblocks; ++base) {
        if (base & a.hmask) continue;
        for (int h = 0; h < hd; ++h) {
            uint64_t j = base;
            for (int i = 0; i < a.nh; ++i)
                if ((h >> i) & 1) j |= uint64_t(1) << a.hq[i];
            idx[h] = j;
        }
        if (!f(idx)) return;
    }
}
}  // namespace

void propagate(const BlockAction &a, BlockSet &d) {
    if (!a.any_couple) return;
    const int hd = 1 << a.nh;
    for_groups(a, d.size(), [&](const uint64_t *idx) {
        bool in[1 << QK_MAX_DENSE_K];
        for (int h = 0; h < hd; ++h) in[h] = d.test(idx[h]);
        for (int ho = 0; ho < hd; ++ho)
            for (int hi = 0; hi < hd; ++hi)
                if (a.couple[size_t(ho) * hd + hi] && in[hi]) d.set(idx[ho]);
        return true;
    });
}

bool closed_under(const BlockAction &a, const BlockSet &s) {
    if (!a.any_couple) return true;
    const int hd = 1 << a.nh;
    bool ok = true;
    for_groups(a, s.size(), [&](const uint64_t *idx) {
        for (int ho = 0; ho < hd && ok; ++ho)
            for (int hi = 0; hi < hd; ++hi)
                if ((a.couple[size_t(ho) * hd + hi] || a.couple[size_t(hi) * hd + ho]) &&
                    s.test(idx[ho]) != s.test(idx[hi])) {
                    ok = false;
                    break;
                }
        return ok;
    });
    return ok;
}

}  // namespace qtask
