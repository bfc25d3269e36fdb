#include "circuit.h"

#include <algorithm>
#include <cmath>

#include "../../include/qtask.h"
#include "lowering.h"

namespace qtask {

long Circuit::index_of(uint64_t level_id) const {
    for (size_t i = 0; i < order_.size(); ++i)
        if (order_[i] == level_id) return long(i);
    return -1;
}

int Circuit::insert_level(uint64_t after, uint64_t *out) {
    if (!out) return QTASK_E_ARG;
    size_t pos = 0;
    if (after != QTASK_FRONT) {
        const long i = index_of(after);
        if (i < 0) return QTASK_E_NOTFOUND;
        pos = size_t(i) + 1;
    }
    Level lv;
    lv.id = next_level_++;
    order_.insert(order_.begin() + long(pos), lv.id);
    levels_.emplace(lv.id, lv);
    touch(pos);
    *out = lv.id;
    return QTASK_OK;
}

int Circuit::remove_level(uint64_t level) {
    const long i = index_of(level);
    if (i < 0) return QTASK_E_NOTFOUND;
    for (uint64_t g : levels_.at(level).gates) gates_.erase(g);
    levels_.erase(level);
    order_.erase(order_.begin() + i);
    touch(size_t(i));
    return QTASK_OK;
}

int Circuit::insert_gate(uint64_t level, int kind, const int32_t *qubits, int nq,
                         const double *params, int np, uint64_t *out) {
    if (!out) return QTASK_E_ARG;
    const int k = kind_arity(kind);
    if (k < 0 || nq != k || !qubits) return QTASK_E_ARG;
    if (np != kind_nparams(kind) || (np > 0 && !params)) return QTASK_E_ARG;
    uint64_t m = 0;
    for (int j = 0; j < nq; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n_) return QTASK_E_ARG;
        const uint64_t bit = uint64_t(1) << qubits[j];
        if (m & bit) return QTASK_E_ARG;
        m |= bit;
    }
    for (int j = 0; j < np; ++j)
        if (!std::isfinite(params[j])) return QTASK_E_ARG;
    const long i = index_of(level);
    if (i < 0) return QTASK_E_NOTFOUND;
    Level &lv = levels_.at(level);
    if (lv.qmask & m) return QTASK_E_CONFLICT;
    Gate g;
    g.id = next_gate_++;
    g.level = level;
    g.kind = kind;
    g.nq = nq;
    for (int j = 0; j < nq; ++j) g.q[j] = qubits[j];
    g.np = np;
    for (int j = 0; j < np; ++j) g.p[j] = params[j];
    gates_.emplace(g.id, g);
    lv.gates.push_back(g.id);
    lv.qmask |= m;
    ++lv.version;
    touch(size_t(i));
    *out = g.id;
    return QTASK_OK;
}

int Circuit::remove_gate(uint64_t gate) {
    auto it = gates_.find(gate);
    if (it == gates_.end()) return QTASK_E_NOTFOUND;
    const Gate &g = it->second;
    Level &lv = levels_.at(g.level);
    for (int j = 0; j < g.nq; ++j) lv.qmask &= ~(uint64_t(1) << g.q[j]);
    lv.gates.erase(std::find(lv.gates.begin(), lv.gates.end(), gate));
    ++lv.version;
    touch(size_t(index_of(g.level)));
    gates_.erase(it);
    return QTASK_OK;
}

int Circuit::level_at(uint64_t index, uint64_t *out) const {
    if (!out) return QTASK_E_ARG;
    if (index >= order_.size()) return QTASK_E_NOTFOUND;
    *out = order_[index];
    return QTASK_OK;
}

}  // namespace qtask
