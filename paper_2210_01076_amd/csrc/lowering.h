// Gate table and lowering of circuit gates to kernel operations.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

#include "kdefs.h"

namespace qtask {

using cd = std::complex<double>;

// A gate lowered to kernel terms.  Qubits are global qubit indices in the
// listed order (q[0] is the high bit of the local matrix index).
struct LGate {
    uint8_t kop = KOP_NONE;  // KOpType
    int nq = 0;
    int q[3] = {-1, -1, -1};
    std::vector<cd> m;       // full 2^nq x 2^nq matrix, row-major, local index order
    std::vector<double> coef;// coefficients the kernel op reads (interleaved re, im)
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
