// Gate table and lowering of circuit gates to kernel operations.
#pragma once
#include <algorithm>
#include <complex>
#include <cstdint>
#include <initializer_list>
#include <vector>

#include "kdefs.h"

namespace qtask {

using cd = std::complex<double>;

// A vector that keeps up to N elements inline (no heap allocation) and moves
// to the heap beyond that.  Lowered gates are copied often while a segment
// is planned; their matrices (4 or 16 entries, 64 for a three-qubit gate)
// and coefficient lists (at most 8) mostly fit inline.
template <typename T, size_t N>
class SmallVec {
public:
    SmallVec() = default;
    SmallVec(std::initializer_list<T> il) { assign(il.begin(), il.end()); }
    SmallVec(const std::vector<T> &v) { assign(v.begin(), v.end()); }
    SmallVec(const SmallVec &o) { assign(o.begin(), o.end()); }
    SmallVec &operator=(const SmallVec &o) {
        if (this != &o) assign(o.begin(), o.end());
        return *this;
    }
    SmallVec &operator=(std::initializer_list<T> il) {
        assign(il.begin(), il.end());
        return *this;
    }
    SmallVec &operator=(const std::vector<T> &v) {
        assign(v.begin(), v.end());
        return *this;
    }
    size_t size() const { return n_; }
    bool empty() const { return n_ == 0; }
    T *data() { return heap_.empty() ? buf_ : heap_.data(); }
    const T *data() const { return heap_.empty() ? buf_ : heap_.data(); }
    T &operator[](size_t i) { return data()[i]; }
    const T &operator[](size_t i) const { return data()[i]; }
    T *begin() { return data(); }
    T *end() { return data() + n_; }
    const T *begin() const { return data(); }
    const T *end() const { return data() + n_; }
    void clear() {
        n_ = 0;
        heap_.clear();
    }
    void push_back(const T &x) {
        if (heap_.empty() && n_ < N) {
            buf_[n_++] = x;
            return;
        }
        if (heap_.empty()) heap_.assign(buf_, buf_ + n_);
        heap_.push_back(x);
        ++n_;
    }

private:
    template <typename It>
    void assign(It b, It e) {
        const size_t k = size_t(e - b);
        heap_.clear();
        if (k <= N) std::copy(b, e, buf_);
        else heap_.assign(b, e);
        n_ = k;
    }
    T buf_[N] = {};
    std::vector<T> heap_;
    size_t n_ = 0;
};

// A gate lowered to kernel terms.  Qubits are global qubit indices in the
// listed order (q[0] is the high bit of the local matrix index).
struct LGate {
    uint8_t kop = KOP_NONE;  // KOpType
    int nq = 0;
    int q[3] = {-1, -1, -1};
    SmallVec<cd, 16> m;       // full 2^nq x 2^nq matrix, row-major, local index order
    SmallVec<double, 8> coef; // coefficients the kernel op reads (interleaved re, im)
    bool diagonal = false;   // matrix is diagonal (decided by kind, never by value)
    bool monomial = false;   // one nonzero per row and column (by kind)
    uint64_t gate_id = 0;    // source gate (0 for ops the planner made)
    uint64_t mask() const {
        uint64_t r = 0;
        for (int j = 0; j < nq; ++j) r |= uint64_t(1) << q[j];
        return r;
    }
    double flops_per_amp() const;  // algorithmic real flops per amplitude
};

// Number of qubits and angle parameters of a qtask_gate_kind; -1 if unknown.
int kind_arity(int kind);
int kind_nparams(int kind);

// The gate's matrix in local-index order (conventions in qtask.h).
std::vector<cd> kind_matrix(int kind, const double *params);

// Lower one gate.  Qubits must already be validated.
LGate lower_gate(int kind, const int *qubits, const double *params, uint64_t gate_id);

// Dense 2^k x 2^k embedding of `g` into the ordered qubit list `qs` (qs[i] is
// bit i of the embedded local index; note: bit 0 = first element).
std::vector<cd> embed(const LGate &g, const std::vector<int> &qs);

}  // namespace qtask
