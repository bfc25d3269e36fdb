// Pass and stage planning for one checkpoint segment.
//
// The paper partitions the state into blocks and runs each gate as tasks over
// the blocks it touches (Section III-C).  On the GPU the same state is swept
// in passes instead: a pass picks b qubits (the c lowest plus up to b-c
// others), loads every tile of 2^b amplitudes spanned by them once into LDS,
// applies every pending gate whose qubits all lie in that set, and writes the
// tile back.  Gates are pulled into a pass as long as no earlier gate left
// for later shares a qubit with them, so the program order of dependent
// gates is kept while independent gates move freely (gates on disjoint
// qubits commute; Section II-A lets parallel gates run in any order).
// Inside a pass the gates are grouped into stages of at most QK_G qubits that
// run on registers; consecutive one-qubit gates on the same qubit are merged
// into one 2x2 matrix (FP64 product), and a stage whose gate list would cost
// more than one dense unitary is fused into that unitary.
#include "planner.h"

#include <algorithm>
#include <cstring>
#include <sstream>
#include <stdexcept>

#include "../../include/qtask.h"

namespace qtask {

namespace {

// Swizzle vectors XOR-ed into the low `swz` bits of an LDS slot for tile bit
// j >= swz.  They are distinct, non-zero and not unit vectors, so any
// choice of lane bits with linearly independent vectors is bank-conflict free.
const uint32_t kSwz4[] = {3, 5, 6, 9, 10, 12, 7, 11, 13, 14, 15};
const uint32_t kSwz5[] = {3, 5, 6, 9, 10, 12, 17, 18, 20, 24, 7, 11};

uint32_t bank_vec(int p, int swz) {
    if (p < swz) return 1u << p;
    return swz == 4 ? kSwz4[p - 4] : kSwz5[p - 5];
}

int popc(uint64_t x) { return __builtin_popcountll(x); }

// LDS banking as the hardware serves a wave (measured with bank-conflict
// counters): a 16-byte read serves 16 lanes per cycle from 256 bytes of
// banks, a 16-byte write 8 lanes from 128 bytes; an 8-byte read 32 lanes from
// 256 bytes, an 8-byte write 16 lanes from 128 bytes.  With slots of
// 2^(4 or 3) bytes, a read is conflict free when the slots of its lane group
// differ in their low `swz` bits and a write when they differ in their low
// swz - 1 bits, i.e. when the bank vectors of the first swz (swz - 1) lane
// bits are linearly independent in those bits.
//
// Order `bits` as lane bits after the fixed lowest lane bits `prefix` (which
// come first, in order): it greedily takes bits whose bank vectors extend an
// independent set, first in the low swz - 1 bits (writes) and then in all
// swz bits (reads), and puts the remaining bits after them in their given
// order.
std::vector<int> lane_order(const std::vector<int> &bits, int swz, const std::vector<int> &prefix = {}) {
    std::vector<int> out(prefix);
    std::vector<int> pool;
    for (int p : bits)
        if (std::find(prefix.begin(), prefix.end(), p) == prefix.end()) pool.push_back(p);
    // independent-set test by GF(2) elimination against the vectors so far
    auto independent = [&](const std::vector<int> &chosen, int p, uint32_t mask) {
        uint32_t basis[32] = {0};
        auto insert = [&](uint32_t v) {
            for (int lead = 31; lead >= 0 && v; --lead)
                if ((v >> lead) & 1) {
                    if (!basis[lead]) { basis[lead] = v; return true; }
                    v ^= basis[lead];
                }
            return false;
        };
        for (int q : chosen) insert(bank_vec(q, swz) & mask);
        return insert(bank_vec(p, swz) & mask);
    };
    for (int level = 0; level < 2; ++level) {
        const int want = level == 0 ? swz - 1 : swz;
        const uint32_t mask = (1u << want) - 1;
        for (size_t i = 0; i < pool.size() && int(out.size()) < want;) {
            if (independent(out, pool[i], mask)) {
                out.push_back(pool[i]);
                pool.erase(pool.begin() + long(i));
            } else {
                ++i;
            }
        }
    }
    out.insert(out.end(), pool.begin(), pool.end());
    return out;
}

bool mergeable(const LGate &g) {
    return g.nq == 1 && (g.kop == KOP_U1 || g.kop == KOP_D1 || g.kop == KOP_A1 || g.kop == KOP_UR ||
                         g.kop == KOP_UX || g.kop == KOP_P1);
}

void set_1q_coef(LGate &g) {
    g.coef.clear();
    auto push = [&](cd z) { g.coef.push_back(z.real()); g.coef.push_back(z.imag()); };
    switch (g.kop) {
    case KOP_D1: push(g.m[0]); push(g.m[3]); break;
    case KOP_P1: push(g.m[3]); break;
    case KOP_A1: push(g.m[1]); push(g.m[2]); break;
    case KOP_UR: for (int i = 0; i < 4; ++i) g.coef.push_back(g.m[i].real()); break;
    default: for (int i = 0; i < 4; ++i) push(g.m[i]); break;
    }
}

// later * earlier for two one-qubit gates on the same qubit.  The class of the
// product follows from the classes of the factors (structural zeros, real
// entries and unit entries stay exact), never from the values.
LGate merge_1q(const LGate &later, const LGate &earlier) {
    LGate r = earlier;
    r.gate_id = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            r.m[i * 2 + j] = later.m[i * 2 + 0] * earlier.m[0 * 2 + j] + later.m[i * 2 + 1] * earlier.m[1 * 2 + j];
    auto diag = [](uint8_t k) { return k == KOP_D1 || k == KOP_P1; };
    const uint8_t a = later.kop, b = earlier.kop;
    if (a == KOP_P1 && b == KOP_P1) {
        r.kop = KOP_P1; r.diagonal = r.monomial = true;
        r.m[0] = cd(1, 0); r.m[1] = r.m[2] = cd(0, 0);
    } else if (diag(a) && diag(b)) {
        r.kop = KOP_D1; r.diagonal = r.monomial = true;
        r.m[1] = r.m[2] = cd(0, 0);
    } else if (a == KOP_A1 && b == KOP_A1) {
        r.kop = KOP_D1; r.diagonal = r.monomial = true;
        r.m[1] = r.m[2] = cd(0, 0);
    } else if ((diag(a) && b == KOP_A1) || (a == KOP_A1 && diag(b))) {
        r.kop = KOP_A1; r.diagonal = false; r.monomial = true;
        r.m[0] = r.m[3] = cd(0, 0);
    } else if (a == KOP_UR && b == KOP_UR) {
        r.kop = KOP_UR; r.diagonal = r.monomial = false;
        for (auto &z : r.m) z = cd(z.real(), 0);
    } else {
        r.kop = KOP_U1; r.diagonal = r.monomial = false;
    }
    set_1q_coef(r);
    return r;
}

// cost units (register FMAs per amplitude) used to decide merges
// A diagonal one-qubit op diag(d0, d1) runs as diag(1, d1/d0), which
// multiplies half the amplitudes instead of all of them; the factors d0 of a
// segment are collected, in plan order, into one scalar that the segment's
// last list stage applies to every amplitude.  A scalar factor commutes with
// every gate, so the segment's result is unchanged up to rounding.
void factor_phases(std::vector<PPass> &passes) {
    // the scalar commutes with every op, so any list stage can hold it: the
    // last one of the segment
    PStage *lastp = nullptr;
    for (auto &ps : passes)
        for (auto &st : ps.stages)
            if (st.U.empty() && !st.mfma) lastp = &st;
    if (!lastp) return;
    PStage &last = *lastp;
    cd g(1, 0);
    bool any = false;
    for (auto &ps : passes)
        for (auto &st : ps.stages) {
            if (!st.U.empty() || st.mfma) continue;
            bool changed = false;
            for (auto &op : st.ops) {
                if (op.kop != KOP_D1) continue;
                const cd d0 = op.m[0];
                g *= d0;
                op.m = {cd(1, 0), cd(0, 0), cd(0, 0), op.m[3] / d0};
                op.kop = KOP_P1;
                set_1q_coef(op);
                changed = any = true;
            }
            if (changed) {
                st.flops = 0;
                for (const auto &op : st.ops) st.flops += op.flops_per_amp();
            }
        }
    if (!any) return;
    LGate gp;
    gp.kop = KOP_GPH;
    gp.nq = 0;
    gp.m = {g};
    gp.diagonal = gp.monomial = true;
    gp.coef = {g.real(), g.imag()};
    last.flops += gp.flops_per_amp();
    last.ops.push_back(gp);
}

double op_cost(const LGate &g) {
    switch (g.kop) {
    case KOP_U1: return 8;
    case KOP_UR: case KOP_UX: case KOP_D1: case KOP_A1: return 4;
    case KOP_P1: return 2;
    default: return 0;
    }
}

std::vector<cd> matmul(const std::vector<cd> &a, const std::vector<cd> &b, int dim) {
    std::vector<cd> c(size_t(dim) * dim, cd(0, 0));
    for (int i = 0; i < dim; ++i)
        for (int k = 0; k < dim; ++k) {
            const cd aik = a[size_t(i) * dim + k];
            if (aik == cd(0, 0)) continue;
            for (int j = 0; j < dim; ++j) c[size_t(i) * dim + j] += aik * b[size_t(k) * dim + j];
        }
    return c;
}

// Below this many qubits a stage's registers are chosen by first fit alone:
// the gain-driven choice saves 5-10% of the stages, which on a small state is
// less device time than the host time it takes to find them (planning sits
// on the critical path of an update).
constexpr int kGainStageQubits = 16;

struct Packer {
    const PlanParams &pp;
    explicit Packer(const PlanParams &p) : pp(p) {}

    // Build the stages of a pass from its ops (program order).
    void pack_stages(PPass &ps, const std::vector<const LGate *> &ops) const {
        const bool dense_mode = pp.fusion == QTASK_FUSE_DENSE;
        const int W = dense_mode ? std::min(pp.fuse_k, pp.b) : QK_G;
        // tile bit of each pass qubit
        int8_t tbit[64];
        for (int q = 0; q < 64; ++q) tbit[q] = -1;
        for (size_t p = 0; p < ps.qlist.size(); ++p) tbit[ps.qlist[p]] = int8_t(p);
        // need: the tile bits an op must have on registers; dep: the tile
        // bits it is ordered on (a free phase needs none, and a qubit it has
        // outside the tile is touched by no other op of the pass but free
        // phases, which commute with it)
        Masks mask64;
        mask64.need.resize(ops.size());
        mask64.dep.resize(ops.size());
        for (size_t i = 0; i < ops.size(); ++i) {
            uint64_t m = 0;
            const bool fp = free_phase(*ops[i]);
            for (int j = 0; j < ops[i]->nq; ++j) {
                if (tbit[ops[i]->q[j]] < 0) {
                    if (!fp) throw std::logic_error("qubit not in pass");
                    continue;
                }
                m |= uint64_t(1) << tbit[ops[i]->q[j]];
            }
            mask64.dep[i] = m;
            mask64.need[i] = fp ? 0 : m;
        }
        std::vector<size_t> rem(ops.size());
        for (size_t i = 0; i < rem.size(); ++i) rem[i] = i;
        // The first stage loads straight from HBM through its own register
        // map, which is coalesced only when its registers avoid the lowest
        // tile bits (those must vary across lanes).  So the first stage is
        // packed from gates above them when there are any; the others wait.
        const uint32_t low_mask = (1u << std::min(coalesce_bits(), pp.b - QK_G)) - 1;
        bool first = true;
        auto fill = [&](uint64_t S) {
            for (int p = pp.b - 1; p >= 0 && popc(S) < W; --p) S |= uint64_t(1) << p;
            return S;
        };
        std::vector<size_t> take, left;
        while (!rem.empty()) {
            // the better of first fit and the gain-driven choice, as for passes
            const uint64_t forbid = first ? low_mask : 0;
            const uint64_t S = pp.n >= kGainStageQubits ? choose_set(mask64, rem, 0, W, forbid, fill)
                                                        : fill(first_fit_set(mask64, rem, 0, W, forbid));
            split_ops(mask64, rem, S, forbid, take, left);
            if (take.empty() && first) {
                first = false;
                continue;  // every pending gate touches the low bits
            }
            first = false;
            if (take.empty()) throw std::logic_error("stage packing made no progress");
            PStage st;
            for (int p = 0; p < pp.b; ++p)
                if ((S >> p) & 1) st.tbits.push_back(p);
            std::vector<int> others;
            for (int p = 0; p < pp.b; ++p)
                if (!((S >> p) & 1)) others.push_back(p);
            st.tpos = lane_order(others, pp.swz);
            // ops, merging consecutive one-qubit gates on the same register qubit
            std::vector<int> last(pp.b, -1);
            st.ops.reserve(take.size());
            bool off_register = false;  // some free phase has a qubit off the registers
            auto on_reg = [&](int q) { return tbit[q] >= 0 && ((S >> tbit[q]) & 1); };
            for (size_t idx : take) {
                const LGate &g = *ops[idx];
                if (mergeable(g) && on_reg(g.q[0])) {
                    const int li = last[tbit[g.q[0]]];
                    if (li >= 0 && mergeable(st.ops[li]) && on_reg(st.ops[li].q[0])) {
                        LGate mg = merge_1q(g, st.ops[li]);
                        if (op_cost(mg) <= op_cost(g) + op_cost(st.ops[li])) {
                            st.ops[li] = mg;
                            continue;
                        }
                    }
                }
                st.ops.push_back(g);
                for (int j = 0; j < g.nq; ++j) {
                    if (tbit[g.q[j]] >= 0) last[tbit[g.q[j]]] = int(st.ops.size()) - 1;
                    off_register = off_register || !on_reg(g.q[j]);
                }
            }
            double fl = 0;
            for (const auto &g : st.ops) fl += g.flops_per_amp();
            st.flops = fl;
            const double dense_fl = 8.0 * (1 << W) - 2;
            bool make_dense = false;
            if (dense_mode) {
                make_dense = true;
                // the matrix-core stage needs whole waves (b >= 10) and at
                // least 16 columns per unitary (b - k >= 4); a 4-qubit
                // unitary on smaller tiles runs on registers instead
                st.mfma = pp.b >= 10 && pp.b - W >= 4;
                if (!st.mfma && W != QK_G) throw std::invalid_argument("dense fusion width needs tile_bits >= 10");
            } else if (pp.fusion == QTASK_FUSE_AUTO && fl > dense_fl && !off_register) {
                make_dense = true;  // dense 16x16 on registers is cheaper than the list
            }
            if (make_dense) {
                std::vector<int> qs;
                for (int p : st.tbits) qs.push_back(ps.qlist[p]);
                const int dim = 1 << int(qs.size());
                std::vector<cd> U(size_t(dim) * dim, cd(0, 0));
                for (int i = 0; i < dim; ++i) U[size_t(i) * dim + i] = 1;
                for (const auto &g : st.ops) U = matmul(embed(g, qs), U, dim);
                st.U = U;
                st.flops = dense_fl;
            }
            ps.stages.push_back(std::move(st));
            rem.swap(left);
        }
    }

    // Every pass has at least one stage, and the lowest lane bits of its
    // first and last stages are the lowest tile bits, which keeps their
    // global loads and stores coalesced.
    // tile bits that must vary across lanes for coalesced 128-byte segments
    int coalesce_bits() const { return pp.dtype == 0 ? 3 : 4; }

    void finish_pass(PPass &ps) const {
        const int lowb = std::min(coalesce_bits(), pp.b - QK_G);
        // tile bits on the lowest physical positions when the pass loads
        // (0, 1, ...) and when it stores (in order of their store position)
        std::vector<int> low_in, low_out;
        for (int q = 0; q < lowb; ++q) {
            for (int p = 0; p < pp.b; ++p)
                if (ps.qlist[size_t(p)] == q) low_in.push_back(p);
            for (int p = 0; p < pp.b; ++p)
                if (ps.out_pos(p) == q) low_out.push_back(p);
        }
        auto touches = [](const PStage &st, const std::vector<int> &bits) {
            for (int p : st.tbits)
                if (std::find(bits.begin(), bits.end(), p) != bits.end()) return true;
            return false;
        };
        // a load- or store-only stage: registers on the highest tile bits
        // that are not among `avoid`
        auto empty_stage = [&](const std::vector<int> &avoid) {
            PStage st;
            for (int p = pp.b - 1; p >= 0 && int(st.tbits.size()) < QK_G; --p)
                if (std::find(avoid.begin(), avoid.end(), p) == avoid.end()) st.tbits.push_back(p);
            std::sort(st.tbits.begin(), st.tbits.end());
            return st;
        };
        // the first stage loads and the last one stores: both must be
        // register stages whose registers avoid the tile bits that must vary
        // across lanes for coalescing; when they are not, a plain load
        // (store) stage goes through LDS instead.  A relabelling pass loads
        // and stores through different global maps, so it needs two stages.
        if (ps.stages.empty() || ps.stages.front().mfma || touches(ps.stages.front(), low_in))
            ps.stages.insert(ps.stages.begin(), empty_stage(low_in));
        if (ps.stages.back().mfma || (ps.stages.size() > 1 && touches(ps.stages.back(), low_out)) ||
            (ps.stages.size() == 1 && ps.relabels()))
            ps.stages.push_back(empty_stage(low_out));
        for (const auto &st : ps.stages) {
            ps.has_mfma = ps.has_mfma || st.mfma;
            ps.has_dense = ps.has_dense || (!st.mfma && !st.U.empty());
        }
        // their lowest lane bits are those tile bits, in order (what
        // coalescing needs); the next ones are chosen for the banks
        for (int which = 0; which < 2; ++which) {
            PStage *st = which == 0 ? &ps.stages.front() : &ps.stages.back();
            const std::vector<int> &lowv = which == 0 ? low_in : low_out;
            std::vector<int> others, low;
            for (int p = 0; p < pp.b; ++p)
                if (std::find(st->tbits.begin(), st->tbits.end(), p) == st->tbits.end()) others.push_back(p);
            for (int p : lowv) {
                if (std::find(others.begin(), others.end(), p) == others.end()) break;
                low.push_back(p);
            }
            st->tpos = lane_order(others, pp.swz, low);
        }
    }

    // Packing a pass (a qubit set of at most b qubits) and packing a stage
    // (a set of at most QK_G tile bits) are the same problem over bit masks:
    // pick a set, then run every pending op whose `need` bits lie in it and
    // that no earlier deferred op blocks.  An op's `dep` bits are the ones it
    // shares an order with: a deferred op blocks every later op that shares
    // a dep bit with it.  need == dep except for the free phases (diagonal
    // ops that run on any set: need is empty).  `forbid` bits may not join
    // the set (the first stage keeps the lowest tile bits on the lanes).
    struct Masks {
        std::vector<uint64_t> need, dep;
    };

    // Ops of `rem` (in order) that a set Q can apply.
    static size_t count_applicable(const Masks &mk, const std::vector<size_t> &rem, uint64_t Q, uint64_t forbid,
                                   size_t limit) {
        uint64_t blocked = forbid;
        size_t cnt = 0;
        for (size_t i = 0; i < rem.size() && i < limit; ++i) {
            const uint64_t d = mk.dep[rem[i]];
            if ((d & blocked) || (mk.need[rem[i]] & ~Q)) blocked |= d;
            else ++cnt;
        }
        return cnt;
    }

    // First fit in program order: each pending op extends the set while it fits.
    static uint64_t first_fit_set(const Masks &mk, const std::vector<size_t> &rem, uint64_t start, int cap,
                                  uint64_t forbid) {
        uint64_t Q = start, blocked = forbid;
        for (size_t idx : rem) {
            const uint64_t d = mk.dep[idx], m = mk.need[idx];
            if (d & blocked) { blocked |= d; continue; }
            if (popc(Q | m) <= cap) Q |= m;
            else blocked |= d;
        }
        return Q;
    }

    // Gain-driven choice: grow the set by the new bits of one of the first
    // pending ops, picking the addition that makes the most ops of the
    // look-ahead window applicable per added bit.
    static uint64_t gain_set(const Masks &mk, const std::vector<size_t> &rem, uint64_t start, int cap,
                             uint64_t forbid) {
        constexpr size_t kWindow = 128, kCands = 8;
        uint64_t Q = start;
        std::vector<uint64_t> cands;
        while (popc(Q) < cap) {
            cands.clear();
            uint64_t blocked = forbid;
            for (size_t i = 0; i < rem.size() && cands.size() < kCands; ++i) {
                const uint64_t m = mk.need[rem[i]], d = mk.dep[rem[i]];
                const uint64_t add = m & ~Q;
                if (!add) continue;
                if (!(d & blocked) && popc(Q | add) <= cap &&
                    std::find(cands.begin(), cands.end(), add) == cands.end())
                    cands.push_back(add);
                blocked |= d;
            }
            if (cands.empty()) break;
            uint64_t best = cands.front();
            double best_v = -1;
            for (uint64_t add : cands) {
                const double v = double(count_applicable(mk, rem, Q | add, forbid, kWindow)) / popc(add);
                if (v > best_v) { best_v = v; best = add; }
            }
            Q |= best;
        }
        return Q;
    }

    // The better of the two sets (more ops applicable), after `fill` tops it up.
    template <typename Fill>
    static uint64_t choose_set(const Masks &mk, const std::vector<size_t> &rem, uint64_t start, int cap,
                               uint64_t forbid, Fill fill) {
        const uint64_t Qf = fill(first_fit_set(mk, rem, start, cap, forbid));
        const size_t nf = count_applicable(mk, rem, Qf, forbid, rem.size());
        if (nf == rem.size()) return Qf;  // nothing left for the other set to win
        const uint64_t Qg = fill(gain_set(mk, rem, start, cap, forbid));
        const size_t ng = count_applicable(mk, rem, Qg, forbid, rem.size());
        return ng > nf ? Qg : Qf;
    }

    // Split rem into the ops the set runs (take) and the rest (left).
    static void split_ops(const Masks &mk, const std::vector<size_t> &rem, uint64_t Q, uint64_t forbid,
                          std::vector<size_t> &take, std::vector<size_t> &left) {
        take.clear();
        left.clear();
        uint64_t blocked = forbid;
        for (size_t idx : rem) {
            const uint64_t d = mk.dep[idx];
            if ((d & blocked) || (mk.need[idx] & ~Q)) { blocked |= d; left.push_back(idx); }
            else take.push_back(idx);
        }
    }

    // A free phase: a diagonal op (phase or diagonal one-qubit matrix) that
    // runs wherever it falls, whichever of its qubits the tile or the stage
    // holds -- the kernel then conditions it on lane bits or on the tile
    // origin.  Not with dense fusion, whose stages fold their ops into one
    // unitary over the stage's own bits.
    bool free_phase(const LGate &g) const {
        return pp.fusion != QTASK_FUSE_DENSE && (g.kop == KOP_P1 || g.kop == KOP_P2 || g.kop == KOP_D1);
    }

    // One pass: its physical tile positions, the ops it runs (already on
    // physical positions) and where it stores each tile bit.
    PPass make_pass(uint64_t pmask, const std::vector<const LGate *> &pops, const std::vector<int> *out_of) const {
        PPass ps;
        ps.qmask = pmask;
        for (int q = 0; q < pp.n; ++q)
            if ((pmask >> q) & 1) ps.qlist.push_back(q);
        if (out_of) {
            for (int q : ps.qlist) ps.out.push_back((*out_of)[size_t(q)]);
            if (ps.out == ps.qlist) ps.out.clear();
        }
        ps.n_gates = int(pops.size());
        pack_stages(ps, pops);
        finish_pass(ps);
        return ps;
    }

    std::vector<PPass> pack_passes(const std::vector<LGate> &ops) const {
        if (pp.relabel) return pack_passes_relabel(ops);
        // keep room for a three-qubit gate on qubits above the low bits, so
        // every pass can take at least the first pending gate
        const int c = std::max(0, std::min(pp.c, pp.b - 3));
        const uint64_t low = (uint64_t(1) << c) - 1;
        Masks mask;
        mask.need.resize(ops.size());
        mask.dep.resize(ops.size());
        for (size_t i = 0; i < ops.size(); ++i) {
            mask.dep[i] = ops[i].mask();
            mask.need[i] = free_phase(ops[i]) ? 0 : mask.dep[i];
        }
        std::vector<size_t> rem(ops.size());
        for (size_t i = 0; i < rem.size(); ++i) rem[i] = i;
        std::vector<PPass> passes;
        std::vector<size_t> take, left;
        take.reserve(ops.size());
        left.reserve(ops.size());
        auto fill = [&](uint64_t Q) {
            for (int q = 0; q < pp.n && popc(Q) < pp.b; ++q) Q |= uint64_t(1) << q;
            return Q;
        };
        while (!rem.empty()) {
            // each pass takes the better of two qubit sets: first fit in
            // program order (which always takes the first pending op) and
            // the gain-driven choice (far fewer passes on layered circuits)
            const uint64_t Q = choose_set(mask, rem, low, pp.b, 0, fill);
            split_ops(mask, rem, Q, 0, take, left);
            if (take.empty()) throw std::logic_error("planner made no progress");
            std::vector<const LGate *> pops;
            pops.reserve(take.size());
            for (size_t idx : take) pops.push_back(&ops[idx]);
            passes.push_back(make_pass(Q, pops, nullptr));
            rem.swap(left);
        }
        return passes;
    }

    // Passes with relabelling.  The sets are chosen over circuit qubits as
    // above, starting from the qubits that sit in the c low positions; the
    // ops are then moved to the physical positions of their qubits.  At the
    // end of a pass the c tile qubits whose next use comes first move into
    // the low positions (those already there keep their slot), and every
    // other tile qubit goes back to its own position when that position is
    // in the tile.  The segment's last pass puts back every qubit whose own
    // position it holds; passes without ops then put back the rest.
    std::vector<PPass> pack_passes_relabel(const std::vector<LGate> &ops) const {
        const int n = pp.n, b = pp.b;
        const int c = std::max(0, std::min(pp.c, pp.b - 3));
        std::vector<int> pos(static_cast<size_t>(n)), occ(static_cast<size_t>(n));  // circuit qubit -> position, position -> qubit
        for (int q = 0; q < n; ++q) pos[size_t(q)] = occ[size_t(q)] = q;
        Masks mask;
        mask.need.resize(ops.size());
        mask.dep.resize(ops.size());
        for (size_t i = 0; i < ops.size(); ++i) {
            mask.dep[i] = ops[i].mask();
            mask.need[i] = free_phase(ops[i]) ? 0 : mask.dep[i];
        }
        std::vector<size_t> rem(ops.size());
        for (size_t i = 0; i < rem.size(); ++i) rem[i] = i;
        std::vector<PPass> passes;
        std::vector<size_t> take, left;
        std::vector<LGate> phys;  // the current pass's ops on physical positions
        constexpr size_t kNever = SIZE_MAX;
        auto fill = [&](uint64_t Q) {
            for (int q = 0; q < n && popc(Q) < b; ++q) Q |= uint64_t(1) << q;
            return Q;
        };
        // assign the tile's qubits to the tile's positions: `hot` (in order)
        // to the low positions, qubits already in a low position keep it;
        // then every other qubit to its own position when that is free,
        // the rest to the remaining positions in ascending order.  With no
        // hot qubits every qubit whose own position is in the tile goes there.
        auto assign = [&](const std::vector<int> &tq, const std::vector<int> &hot, std::vector<int> &newpos) {
            std::vector<int> freep;
            for (int q : tq) freep.push_back(pos[size_t(q)]);
            std::sort(freep.begin(), freep.end());
            auto take_pos = [&](int p) { freep.erase(std::find(freep.begin(), freep.end(), p)); };
            std::vector<char> done(static_cast<size_t>(n), 0);
            if (hot.empty())
                for (int q : tq)
                    if (std::find(freep.begin(), freep.end(), q) != freep.end()) {
                        newpos[size_t(q)] = q;
                        take_pos(q);
                        done[size_t(q)] = 1;
                    }
            for (int q : hot)
                if (pos[size_t(q)] < c) { newpos[size_t(q)] = pos[size_t(q)]; take_pos(pos[size_t(q)]); done[size_t(q)] = 1; }
            for (int q : hot)
                if (!done[size_t(q)]) {
                    const int p = freep.front();  // a low position (the low ones are all in the tile)
                    newpos[size_t(q)] = p;
                    take_pos(p);
                    done[size_t(q)] = 1;
                }
            for (int q : tq)
                if (!done[size_t(q)] && std::find(freep.begin(), freep.end(), q) != freep.end()) {
                    newpos[size_t(q)] = q;
                    take_pos(q);
                    done[size_t(q)] = 1;
                }
            for (int q : tq)
                if (!done[size_t(q)]) {
                    newpos[size_t(q)] = freep.front();
                    take_pos(freep.front());
                }
        };
        auto apply = [&](const std::vector<int> &tq, const std::vector<int> &newpos, std::vector<int> &out_of) {
            // out_of: physical position before -> after, for the tile's positions
            for (int q : tq) out_of[size_t(pos[size_t(q)])] = newpos[size_t(q)];
            for (int q : tq) {
                pos[size_t(q)] = newpos[size_t(q)];
                occ[size_t(newpos[size_t(q)])] = q;
            }
        };
        std::vector<int> newpos(static_cast<size_t>(n)), out_of(static_cast<size_t>(n));
        while (!rem.empty()) {
            uint64_t start = 0;
            for (int p = 0; p < c; ++p) start |= uint64_t(1) << occ[size_t(p)];
            const uint64_t Q = choose_set(mask, rem, start, b, 0, fill);
            split_ops(mask, rem, Q, 0, take, left);
            if (take.empty()) throw std::logic_error("planner made no progress");
            std::vector<int> tq;
            uint64_t pmask = 0;
            for (int q = 0; q < n; ++q)
                if ((Q >> q) & 1) {
                    tq.push_back(q);
                    pmask |= uint64_t(1) << pos[size_t(q)];
                }
            phys.clear();
            phys.reserve(take.size());
            for (size_t idx : take) {
                LGate g = ops[idx];
                for (int j = 0; j < g.nq; ++j) g.q[j] = pos[size_t(g.q[j])];
                phys.push_back(std::move(g));
            }
            std::vector<const LGate *> pops;
            for (const LGate &g : phys) pops.push_back(&g);
            rem.swap(left);
            // where the tile's qubits go
            std::vector<int> hot;
            if (!rem.empty()) {
                std::vector<size_t> next(static_cast<size_t>(n), kNever);
                size_t found = 0;
                for (size_t k = 0; k < rem.size() && found < tq.size(); ++k) {
                    const LGate &g = ops[rem[k]];
                    if (!mask.need[rem[k]]) continue;  // a free phase needs no tile position
                    for (int j = 0; j < g.nq; ++j)
                        if (next[size_t(g.q[j])] == kNever && ((Q >> g.q[j]) & 1)) {
                            next[size_t(g.q[j])] = k;
                            ++found;
                        }
                }
                hot = tq;
                std::stable_sort(hot.begin(), hot.end(), [&](int x, int y) {
                    if (next[size_t(x)] != next[size_t(y)]) return next[size_t(x)] < next[size_t(y)];
                    return (pos[size_t(x)] < c) > (pos[size_t(y)] < c);
                });
                hot.resize(size_t(c));
            }
            assign(tq, hot, newpos);
            apply(tq, newpos, out_of);
            passes.push_back(make_pass(pmask, pops, &out_of));
        }
        // passes without ops put back the qubits still away from their own
        // position: each takes the low positions plus, qubit by qubit, the
        // current and the own position of displaced qubits while they fit
        for (int guard = 0; guard < 4 * n; ++guard) {
            std::vector<int> away;
            for (int q = 0; q < n; ++q)
                if (pos[size_t(q)] != q) away.push_back(q);
            if (away.empty()) return passes;
            uint64_t pmask = (uint64_t(1) << c) - 1;
            for (int q : away) {
                const uint64_t add = (uint64_t(1) << pos[size_t(q)]) | (uint64_t(1) << q);
                if (popc(pmask | add) <= b) pmask |= add;
            }
            for (int p = 0; p < n && popc(pmask) < b; ++p) pmask |= uint64_t(1) << p;
            std::vector<int> tq;
            for (int p = 0; p < n; ++p)
                if ((pmask >> p) & 1) tq.push_back(occ[size_t(p)]);
            std::sort(tq.begin(), tq.end());
            assign(tq, {}, newpos);
            apply(tq, newpos, out_of);
            passes.push_back(make_pass(pmask, {}, &out_of));
        }
        throw std::logic_error("relabelling did not return to the plain layout");
    }
};

// A matrix-core stage's operand in the order the kernel's lanes read it.
// The stage multiplies by the real block matrix M = [[Ur, -Ui], [Ui, Ur]]
// (2^(k+1) rows and columns) with 16x16x4 matrix instructions: in inner
// step s, lane l of a wave holds, for row block rb, the element of M at row
// 16 rb + l % 16 and column 4 s + l / 16.  That element is stored at
// (s * 64 + l) * RB + rb (RB = 2^(k+1) / 16 row blocks), so each lane reads
// the RB values of a step as one contiguous vector.  Values are rounded
// once from the FP64 unitary.  Returns the count written (4 * 4^k).
constexpr size_t kMfmaAlign = 16;  // operand offset alignment, in values

template <typename R>
size_t pack_mfma_operand(const std::vector<cd> &U, int k, R *out) {
    const int dim = 1 << k, mr = 2 * dim, rb_n = mr / 16, steps = mr / 4;
    for (int s = 0; s < steps; ++s)
        for (int l = 0; l < 64; ++l)
            for (int rb = 0; rb < rb_n; ++rb) {
                const int row = 16 * rb + (l & 15), col = 4 * s + (l >> 4);
                const cd z = U[size_t(row & (dim - 1)) * dim + (col & (dim - 1))];
                const bool top = row < dim, right = col >= dim;
                double v = top == right ? z.imag() : z.real();  // Ui in the off-diagonal blocks
                if (top && right) v = -v;
                out[size_t(s * 64 + l) * rb_n + rb] = R(v);
            }
    return size_t(mr) * mr;
}

template <typename R>
void pack_blob(SegmentPlan &sp) {
    const PlanParams &pp = sp.pp;
    const int b = pp.b, G = QK_G;
    const int n_thr = b - G;
    size_t n_stage = 0, n_op = 0, n_coef = 0;
    for (const auto &ps : sp.passes)
        for (const auto &st : ps.stages) {
            ++n_stage;
            if (st.mfma) n_coef += kMfmaAlign + 2 * st.U.size() * 2;  // block form, aligned
            else if (!st.U.empty()) { n_op += 1; n_coef += st.U.size() * 2; }
            else {
                for (const auto &g : st.ops) { ++n_op; n_coef += g.coef.size(); }
                ++n_op;  // room for the stage's KOP_PHI
            }
        }
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t bytes_pass = align(sp.passes.size() * sizeof(KPass));
    const size_t bytes_stage = align(n_stage * sizeof(KStage));
    // one spare record: the kernel reads the record after a stage's last op
    const size_t bytes_op = align((n_op + 1) * sizeof(KOp));
    const size_t bytes_coef = align(std::max<size_t>(n_coef, 1) * sizeof(R));
    sp.off_stage = bytes_pass;
    sp.off_op = bytes_pass + bytes_stage;
    sp.off_coef = sp.off_op + bytes_op;
    sp.blob.assign(sp.off_coef + bytes_coef, 0);
    KPass *kp = reinterpret_cast<KPass *>(sp.blob.data());
    KStage *ks = reinterpret_cast<KStage *>(sp.blob.data() + sp.off_stage);
    KOp *ko = reinterpret_cast<KOp *>(sp.blob.data() + sp.off_op);
    R *kc = reinterpret_cast<R *>(sp.blob.data() + sp.off_coef);
    size_t si = 0, oi = 0, ci = 0;
    auto phys = [&](int p) { return lds_phys(1u << p, pp.swz); };
    for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
        const PPass &ps = sp.passes[pi];
        KPass &P = kp[pi];
        std::memset(&P, 0, sizeof(P));
        auto goff = [&](int p) { return uint64_t(1) << ps.qlist[p]; };
        int k = 0;
        for (int q = 0; q < pp.n; ++q) {
            if ((ps.qmask >> q) & 1) continue;
            if (q == 0 || ((ps.qmask >> (q - 1)) & 1)) {
                if (P.n_runs >= QK_MAX_RUNS) throw std::logic_error("too many non-tile runs");
                P.run[P.n_runs++] = uint32_t(k) | uint32_t(q) << 16;
            }
            P.run[P.n_runs - 1] += 1u << 8;
            P.nonq_pos[k++] = uint8_t(q);
        }
        P.n_nonq = uint32_t(k);
        P.n_thr = uint32_t(n_thr);
        P.stage_begin = uint32_t(si);
        P.stage_count = uint32_t(ps.stages.size());
        // the first stage loads tile bit p from position qlist[p], the last
        // one stores it to out_pos(p) (the same unless the pass relabels)
        auto goff_out = [&](int p) { return uint64_t(1) << ps.out_pos(p); };
        for (size_t sti = 0; sti < ps.stages.size(); ++sti) {
            const PStage &st = ps.stages[sti];
            KStage &S = ks[si++];
            std::memset(&S, 0, sizeof(S));
            const int W = int(st.tbits.size());
            const bool store = sti + 1 == ps.stages.size();
            if (!st.mfma) {
                for (int j = 0; j < G; ++j) S.g_bit[j] = store ? goff_out(st.tbits[j]) : goff(st.tbits[j]);
                for (int j = 0; j < n_thr; ++j) S.g_thr[j] = store ? goff_out(st.tpos[j]) : goff(st.tpos[j]);
            }
            if (st.mfma) {
                S.kind = KSTAGE_MFMA;
                S.k = uint32_t(W);
                S.n_col_bits = uint32_t(b - W);
                for (int r = 0; r < (1 << W); ++r) {
                    uint32_t o = 0;
                    for (int j = 0; j < W; ++j)
                        if ((r >> j) & 1) o ^= phys(st.tbits[j]);
                    S.row_off[r] = o;
                }
                for (int j = 0; j < b - W; ++j) S.col_off[j] = phys(st.tpos[j]);
                ci = (ci + kMfmaAlign - 1) / kMfmaAlign * kMfmaAlign;
                S.coef = uint32_t(ci);
                ci += pack_mfma_operand(st.U, W, kc + ci);
                S.op_begin = uint32_t(oi);
                S.op_count = 0;
                continue;
            }
            S.kind = KSTAGE_LIST;
            for (int j = 0; j < G; ++j) S.reg_bit[j] = phys(st.tbits[j]);
            for (int j = 0; j < n_thr; ++j) S.thr_off[j] = phys(st.tpos[j]);
            S.op_begin = uint32_t(oi);
            auto reg_of = [&](int q) {
                const int tb = [&] {
                    for (size_t p = 0; p < ps.qlist.size(); ++p)
                        if (ps.qlist[p] == q) return int(p);
                    return -1;
                }();
                for (int j = 0; j < G; ++j)
                    if (st.tbits[j] == tb) return j;
                throw std::logic_error("op qubit outside its stage");
            };
            if (!st.U.empty()) {
                KOp &o = ko[oi++];
                o.type = KOP_DENSE;
                o.a = o.b = o.c = 0;
                o.coef = uint32_t(ci);
                for (const cd &z : st.U) { kc[ci++] = R(z.real()); kc[ci++] = R(z.imag()); }
            } else {
                // where a qubit sits in the stage: register bit j (j), lane
                // bit k (KPC_LANE + k), or off the tile (KPC_ORIGIN + its
                // position: a bit of the tile origin)
                auto code_of = [&](int q) -> uint8_t {
                    int tb = -1;
                    for (size_t p = 0; p < ps.qlist.size(); ++p)
                        if (ps.qlist[p] == q) tb = int(p);
                    if (tb < 0) return uint8_t(KPC_ORIGIN + q);
                    for (int j = 0; j < G; ++j)
                        if (st.tbits[j] == tb) return uint8_t(j);
                    for (int k = 0; k < n_thr; ++k)
                        if (st.tpos[k] == tb) return uint8_t(KPC_LANE + k);
                    throw std::logic_error("op qubit outside its pass");
                };
                // Phases with no qubit on the registers (and the global
                // phase) scale whole lanes: they commute with every op of the
                // stage, so they go last, into the lane's pending factor,
                // which one KOP_PHI then applies.
                std::vector<const LGate *> lane_phases;
                for (const LGate &g : st.ops) {
                    if (lane_phase(ps, st, g)) {
                        if (g.kop != KOP_GPH && g.kop != KOP_P1 && g.kop != KOP_P2)
                            throw std::logic_error("off-register op is no phase");
                        lane_phases.push_back(&g);
                        continue;
                    }
                    bool regs = true;
                    for (int j = 0; j < g.nq; ++j) regs = regs && code_of(g.q[j]) < G;
                    KOp &o = ko[oi++];
                    o.coef = uint32_t(ci);
                    if (!regs) {
                        // a free phase with one qubit on the registers and
                        // the other on a lane or off the tile
                        if (g.kop != KOP_P2) throw std::logic_error("off-register op is no phase");
                        const uint8_t c0 = code_of(g.q[0]), c1 = code_of(g.q[1]);
                        o.type = KOP_PC;
                        o.a = c0 < G ? c0 : c1;
                        o.b = c0 < G ? c1 : c0;
                        o.c = 0;
                        for (double v : g.coef) kc[ci++] = R(v);
                        continue;
                    }
                    o.type = g.kop;
                    o.a = g.nq > 0 ? uint8_t(reg_of(g.q[0])) : 0;
                    o.b = g.nq > 1 ? uint8_t(reg_of(g.q[1])) : 0;
                    o.c = g.nq > 2 ? uint8_t(reg_of(g.q[2])) : 0;
                    if (g.kop == KOP_CCX && o.a > o.b) std::swap(o.a, o.b);
                    for (double v : g.coef) kc[ci++] = R(v);
                }
                for (const LGate *g : lane_phases) {
                    KOp &o = ko[oi++];
                    o.type = KOP_PCL;
                    o.a = g->nq > 0 ? code_of(g->q[0]) : uint8_t(KPC_NONE);
                    o.b = g->nq > 1 ? code_of(g->q[1]) : uint8_t(KPC_NONE);
                    o.c = 0;
                    o.coef = uint32_t(ci);
                    for (double v : g->coef) kc[ci++] = R(v);
                }
                if (!lane_phases.empty()) {
                    KOp &o = ko[oi++];
                    o.type = KOP_PHI;
                    o.a = o.b = o.c = 0;
                    o.coef = uint32_t(ci);
                }
            }
            S.op_count = uint32_t(oi) - S.op_begin;
        }
    }
}


}  // namespace

bool lane_phase(const PPass &ps, const PStage &st, const LGate &g) {
    if (g.kop == KOP_GPH) return true;
    if (g.nq == 0 || !st.U.empty() || st.mfma) return false;
    for (int j = 0; j < g.nq; ++j)
        for (int tb : st.tbits)
            if (ps.qlist[size_t(tb)] == g.q[j]) return false;
    return true;
}

uint32_t lds_phys(uint32_t l, int swz) {
    uint32_t x = l;
    for (int j = swz; j < QK_MAX_TILE_BITS; ++j)
        if ((l >> j) & 1) x ^= bank_vec(j, swz);
    return x;
}

uint64_t segment_hash(const std::vector<LGate> &ops, const PlanParams &pp) {
    // the plan cache is keyed by this value, so it mixes every bit of the
    // kinds, qubits and matrices
    auto mix = hash_mix;
    uint64_t h = 0x243f6a8885a308d3ull;
    const int64_t params[8] = {pp.n, pp.b, pp.c, pp.dtype, pp.fusion, pp.fuse_k, pp.swz, pp.relabel};
    for (int64_t v : params) h = mix(h, uint64_t(v));
    for (const auto &g : ops) {
        h = mix(h, uint64_t(g.kop) | (uint64_t(uint8_t(g.nq)) << 8) | (uint64_t(uint16_t(g.q[0])) << 16) |
                       (uint64_t(uint16_t(g.q[1])) << 32) | (uint64_t(uint16_t(g.q[2])) << 48));
        for (const cd &z : g.m) {
            uint64_t re, im;
            const double r = z.real(), i = z.imag();
            std::memcpy(&re, &r, 8);
            std::memcpy(&im, &i, 8);
            h = mix(mix(h, re), im);
        }
    }
    return h;
}

SegmentPlan plan_segment(const std::vector<LGate> &ops, const PlanParams &pp, uint64_t hash) {
    if (pp.b < QK_MIN_TILE_BITS || pp.b > QK_MAX_TILE_BITS || pp.b > pp.n || pp.c < 0 || pp.c > pp.b)
        throw std::invalid_argument("plan parameters");
    SegmentPlan sp;
    sp.pp = pp;
    Packer pk(pp);
    sp.passes = pk.pack_passes(ops);
    factor_phases(sp.passes);
    if (sp.passes.empty()) {
        // a segment without gates still carries the state across its
        // boundary (restore, checkpoint write, norm): one pass, one empty stage
        PPass ps;
        for (int q = 0; q < pp.b; ++q) {
            ps.qlist.push_back(q);
            ps.qmask |= uint64_t(1) << q;
        }
        pk.finish_pass(ps);
        sp.passes.push_back(ps);
    }
    sp.n_gates = ops.size();
    for (const auto &ps : sp.passes)
        for (const auto &st : ps.stages) sp.flops_per_amp += st.flops;
    if (pp.dtype == 0) pack_blob<double>(sp);
    else pack_blob<float>(sp);
    sp.hash = hash ? hash : segment_hash(ops, pp);
    return sp;
}

std::string validate_plan(const SegmentPlan &sp) {
    const PlanParams &pp = sp.pp;
    const int b = pp.b, G = QK_G, n_thr = b - G;
    const uint32_t tile = 1u << b;
    std::ostringstream err;
    const KPass *kp = reinterpret_cast<const KPass *>(sp.blob.data());
    const KStage *ks = reinterpret_cast<const KStage *>(sp.blob.data() + sp.off_stage);
    size_t gates = 0;
    for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
        const KPass &P = kp[pi];
        const PPass &ps = sp.passes[pi];
        gates += size_t(ps.n_gates);
        if (int(ps.qlist.size()) != b) { err << "pass " << pi << ": qlist size"; return err.str(); }
        for (int q = 0; q < std::max(0, std::min(pp.c, pp.b - 3)); ++q)
            if (ps.qlist[q] != q) { err << "pass " << pi << ": low bits"; return err.str(); }
        if (P.stage_count < 1) { err << "pass " << pi << ": no stage"; return err.str(); }
        {
            // the deposit runs must send tile-index bit k to nonq_pos[k], in order
            uint32_t k = 0;
            for (uint32_t r = 0; r < P.n_runs; ++r) {
                const uint32_t src = P.run[r] & 0xff, len = (P.run[r] >> 8) & 0xff, dst = P.run[r] >> 16;
                if (src != k || len == 0) { err << "pass " << pi << ": deposit runs"; return err.str(); }
                for (uint32_t j = 0; j < len; ++j, ++k)
                    if (k >= P.n_nonq || P.nonq_pos[k] != dst + j) { err << "pass " << pi << ": deposit runs"; return err.str(); }
            }
            if (k != P.n_nonq || P.n_nonq != uint32_t(pp.n - b)) { err << "pass " << pi << ": deposit runs"; return err.str(); }
        }
        for (uint32_t which : {P.stage_begin, P.stage_begin + P.stage_count - 1}) {
            const KStage &S = ks[which];
            if (S.kind != KSTAGE_LIST) { err << "pass " << pi << ": first/last stage must be a list stage"; return err.str(); }
            std::vector<uint64_t> offs;
            uint64_t gmask = 0;
            for (uint32_t t = 0; t < (1u << n_thr); ++t) {
                uint64_t gt = 0;
                for (int k = 0; k < n_thr; ++k)
                    if ((t >> k) & 1) gt |= S.g_thr[k];
                for (int i = 0; i < QK_NREG; ++i) {
                    uint64_t gr = 0;
                    for (int j = 0; j < G; ++j)
                        if ((i >> j) & 1) {
                            if (gr & S.g_bit[j]) { err << "pass " << pi << ": register bits overlap"; return err.str(); }
                            gr |= S.g_bit[j];
                        }
                    if (gt & gr) { err << "pass " << pi << ": global map overlap"; return err.str(); }
                    offs.push_back(gt | gr);
                    gmask |= gt | gr;
                }
            }
            std::sort(offs.begin(), offs.end());
            if (std::unique(offs.begin(), offs.end()) != offs.end()) { err << "pass " << pi << ": global map not one-to-one"; return err.str(); }
            if (gmask != ps.qmask) { err << "pass " << pi << ": global mask"; return err.str(); }
        }
        for (uint32_t s = 0; s < P.stage_count; ++s) {
            const KStage &S = ks[P.stage_begin + s];
            const PStage &st = ps.stages[s];
            std::vector<uint8_t> seen2(tile, 0);
            if (S.kind == KSTAGE_MFMA) {
                for (uint32_t col = 0; col < (1u << S.n_col_bits); ++col) {
                    uint32_t co = 0;
                    for (uint32_t j = 0; j < S.n_col_bits; ++j)
                        if ((col >> j) & 1) co ^= S.col_off[j];
                    for (uint32_t r = 0; r < (1u << S.k); ++r) {
                        const uint32_t sl = co ^ S.row_off[r];
                        if (sl >= tile || seen2[sl]++) { err << "pass " << pi << " stage " << s << ": mfma map"; return err.str(); }
                    }
                }
            } else {
                for (uint32_t t = 0; t < (1u << n_thr); ++t) {
                    uint32_t bt = 0;
                    for (int k = 0; k < n_thr; ++k)
                        if ((t >> k) & 1) bt ^= S.thr_off[k];
                    for (int i = 0; i < QK_NREG; ++i) {
                        uint32_t ro = 0;
                        for (int j = 0; j < G; ++j)
                            if ((i >> j) & 1) ro ^= S.reg_bit[j];
                        const uint32_t sl = bt ^ ro;
                        if (sl >= tile || seen2[sl]++) { err << "pass " << pi << " stage " << s << ": reg map"; return err.str(); }
                    }
                }
            }
            uint64_t sq = 0;
            for (int p : st.tbits) sq |= uint64_t(1) << ps.qlist[p];
            for (const auto &g : st.ops)
                if ((g.mask() & ~sq) != 0 && g.kop != KOP_P1 && g.kop != KOP_P2) {
                    err << "pass " << pi << " stage " << s << ": op outside stage";
                    return err.str();
                }
        }
    }
    if (gates != sp.n_gates) { err << "gate count " << gates << " != " << sp.n_gates; return err.str(); }
    return "";
}

// The blob records of pass pi as the kernel reads them: deposit runs, and
// per stage the LDS maps, the global maps, the op records and (matrix-core
// stages) the row and column slots.
static void blob_json(std::ostringstream &o, const SegmentPlan &sp, size_t pi) {
    const KPass &P = reinterpret_cast<const KPass *>(sp.blob.data())[pi];
    const KStage *ks = reinterpret_cast<const KStage *>(sp.blob.data() + sp.off_stage);
    const KOp *ko = reinterpret_cast<const KOp *>(sp.blob.data() + sp.off_op);
    auto arr = [&](const char *name, auto *v, size_t len) {
        o << ",\"" << name << "\":[";
        for (size_t i = 0; i < len; ++i) o << (i ? "," : "") << uint64_t(v[i]);
        o << "]";
    };
    o << "{\"n_thr\":" << P.n_thr;
    arr("runs", P.run, P.n_runs);
    o << ",\"stages\":[";
    for (uint32_t s = 0; s < P.stage_count; ++s) {
        const KStage &S = ks[P.stage_begin + s];
        o << (s ? "," : "") << "{\"kind\":" << S.kind << ",\"k\":" << S.k << ",\"coef\":" << S.coef;
        arr("reg_bit", S.reg_bit, QK_G);
        arr("thr_off", S.thr_off, QK_MAX_THR_BITS);
        arr("g_bit", S.g_bit, QK_G);
        arr("g_thr", S.g_thr, QK_MAX_THR_BITS);
        arr("row_off", S.row_off, size_t(1) << std::min<uint32_t>(S.k, QK_MAX_DENSE_K));
        arr("col_off", S.col_off, S.n_col_bits);
        o << ",\"ops\":[";
        for (uint32_t k = 0; k < S.op_count; ++k) {
            const KOp &op = ko[S.op_begin + k];
            o << (k ? "," : "") << "[" << int(op.type) << "," << int(op.a) << "," << int(op.b) << "," << int(op.c)
              << "," << op.coef << "]";
        }
        o << "]}";
    }
    o << "]}";
}

std::string plan_json(const SegmentPlan &sp, bool with_matrices) {
    std::ostringstream o;
    o.precision(17);
    o << "{\"b\":" << sp.pp.b << ",\"c\":" << sp.pp.c << ",\"n\":" << sp.pp.n << ",\"dtype\":" << sp.pp.dtype
      << ",\"fusion\":" << sp.pp.fusion << ",\"fuse_k\":" << sp.pp.fuse_k << ",\"gates\":" << sp.n_gates
      << ",\"flops_per_amp\":" << sp.flops_per_amp << ",\"check\":\"" << validate_plan(sp) << "\",\"passes\":[";
    for (size_t pi = 0; pi < sp.passes.size(); ++pi) {
        const PPass &ps = sp.passes[pi];
        if (pi) o << ",";
        o << "{\"qubits\":[";
        for (size_t i = 0; i < ps.qlist.size(); ++i) o << (i ? "," : "") << ps.qlist[i];
        o << "],\"out\":[";
        for (int p = 0; p < int(ps.qlist.size()); ++p) o << (p ? "," : "") << ps.out_pos(p);
        o << "],\"gates\":" << ps.n_gates << ",\"stages\":[";
        for (size_t si = 0; si < ps.stages.size(); ++si) {
            const PStage &st = ps.stages[si];
            if (si) o << ",";
            o << "{\"qubits\":[";
            for (size_t i = 0; i < st.tbits.size(); ++i) o << (i ? "," : "") << ps.qlist[st.tbits[i]];
            o << "],\"reg_tile_bits\":[";
            for (size_t i = 0; i < st.tbits.size(); ++i) o << (i ? "," : "") << st.tbits[i];
            o << "],\"lane_tile_bits\":[";
            for (size_t i = 0; i < st.tpos.size(); ++i) o << (i ? "," : "") << st.tpos[i];
            o << "],\"mfma\":" << (st.mfma ? "true" : "false") << ",\"dense\":" << (st.U.empty() ? "false" : "true")
              << ",\"flops_per_amp\":" << st.flops << ",\"ops\":[";
            for (size_t k = 0; k < st.ops.size(); ++k) {
                const LGate &g = st.ops[k];
                if (k) o << ",";
                o << "{\"kop\":" << int(g.kop) << ",\"gate\":" << g.gate_id << ",\"q\":[";
                for (int j = 0; j < g.nq; ++j) o << (j ? "," : "") << g.q[j];
                o << "]";
                if (with_matrices) {
                    o << ",\"m\":[";
                    for (size_t z = 0; z < g.m.size(); ++z)
                        o << (z ? "," : "") << "[" << g.m[z].real() << "," << g.m[z].imag() << "]";
                    o << "]";
                }
                o << "}";
            }
            o << "]";
            if (with_matrices && !st.U.empty()) {
                o << ",\"U\":[";
                for (size_t z = 0; z < st.U.size(); ++z)
                    o << (z ? "," : "") << "[" << st.U[z].real() << "," << st.U[z].imag() << "]";
                o << "]";
            }
            o << "}";
        }
        o << "]";
        if (with_matrices) {
            o << ",\"kernel\":";
            blob_json(o, sp, pi);
        }
        o << "}";
    }
    o << "]";
    if (with_matrices) {
        // the coefficient array (as the kernel reads it, in the session dtype)
        const size_t ncoef = (sp.blob.size() - sp.off_coef) / (sp.pp.dtype == 0 ? sizeof(double) : sizeof(float));
        o << ",\"coefs\":[";
        for (size_t i = 0; i < ncoef; ++i) {
            const double v = sp.pp.dtype == 0 ? reinterpret_cast<const double *>(sp.blob.data() + sp.off_coef)[i]
                                              : double(reinterpret_cast<const float *>(sp.blob.data() + sp.off_coef)[i]);
            o << (i ? "," : "") << v;
        }
        o << "]";
    }
    o << "}";
    return o.str();
}

}  // namespace qtask
