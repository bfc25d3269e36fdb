// Gate table of the library (written independently of the test oracle; the
// conventions are the ones stated in qtask.h) and lowering to kernel ops.
//
// Gate modes follow the paper's split (Section III-C): gates that create no
// superposition (CNOT, diagonal and permutation gates) become exact exchanges
// or phase scalings, the others go through a small dense matrix.  The class
// of a gate is decided by its kind only, never by the value of an angle.
#include "lowering.h"

#include <cmath>
#include <stdexcept>

#include "../../include/qtask.h"

namespace qtask {

int kind_arity(int kind) {
    switch (kind) {
    case QTASK_H: case QTASK_X: case QTASK_Y: case QTASK_Z: case QTASK_S: case QTASK_SDG:
    case QTASK_T: case QTASK_TDG: case QTASK_RX: case QTASK_RY: case QTASK_RZ:
        return 1;
    case QTASK_CX: case QTASK_CZ: case QTASK_SWAP: case QTASK_CP:
        return 2;
    case QTASK_CCX:
        return 3;
    default:
        return -1;
    }
}

int kind_nparams(int kind) {
    switch (kind) {
    case QTASK_RX: case QTASK_RY: case QTASK_RZ: case QTASK_CP:
        return 1;
    default:
        return kind_arity(kind) < 0 ? -1 : 0;
    }
}

std::vector<cd> kind_matrix(int kind, const double *p) {
    const int k = kind_arity(kind);
    if (k < 0) throw std::invalid_argument("gate kind");
    const int dim = 1 << k;
    std::vector<cd> m(size_t(dim) * dim, cd(0, 0));
    auto at = [&](int r, int c) -> cd & { return m[size_t(r) * dim + c]; };
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (kind) {
    case QTASK_H: at(0, 0) = r2; at(0, 1) = r2; at(1, 0) = r2; at(1, 1) = -r2; break;
    case QTASK_X: at(0, 1) = 1; at(1, 0) = 1; break;
    case QTASK_Y: at(0, 1) = cd(0, -1); at(1, 0) = cd(0, 1); break;
    case QTASK_Z: at(0, 0) = 1; at(1, 1) = -1; break;
    case QTASK_S: at(0, 0) = 1; at(1, 1) = cd(0, 1); break;
    case QTASK_SDG: at(0, 0) = 1; at(1, 1) = cd(0, -1); break;
    case QTASK_T: at(0, 0) = 1; at(1, 1) = cd(r2, r2); break;
    case QTASK_TDG: at(0, 0) = 1; at(1, 1) = cd(r2, -r2); break;
    case QTASK_RX: {
        const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        at(0, 0) = c; at(0, 1) = cd(0, -s); at(1, 0) = cd(0, -s); at(1, 1) = c; break;
    }
    case QTASK_RY: {
        const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        at(0, 0) = c; at(0, 1) = -s; at(1, 0) = s; at(1, 1) = c; break;
    }
    case QTASK_RZ: {
        const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        at(0, 0) = cd(c, -s); at(1, 1) = cd(c, s); break;
    }
    case QTASK_CX: at(0, 0) = 1; at(1, 1) = 1; at(2, 3) = 1; at(3, 2) = 1; break;
    case QTASK_CZ: at(0, 0) = 1; at(1, 1) = 1; at(2, 2) = 1; at(3, 3) = -1; break;
    case QTASK_SWAP: at(0, 0) = 1; at(1, 2) = 1; at(2, 1) = 1; at(3, 3) = 1; break;
    case QTASK_CP:
        at(0, 0) = 1; at(1, 1) = 1; at(2, 2) = 1; at(3, 3) = cd(std::cos(p[0]), std::sin(p[0])); break;
    case QTASK_CCX:
        for (int i = 0; i < 6; ++i) at(i, i) = 1;
        at(6, 7) = 1; at(7, 6) = 1; break;
    }
    return m;
}

static void push(SmallVec<double, 8> &v, cd z) {
    v.push_back(z.real());
    v.push_back(z.imag());
}

double LGate::flops_per_amp() const {
    // real flops per amplitude as executed (complex multiply = 6 flops,
    // complex add = 2; a real-by-complex multiply = 2)
    switch (kop) {
    case KOP_U1: return 14;
    case KOP_UR: case KOP_UX: return 6;
    case KOP_D1: case KOP_A1: return 6;
    case KOP_P1: return 3;        // half of the amplitudes get a phase
    case KOP_P2: return 1.5;      // a quarter of the amplitudes get a phase
    case KOP_GPH: return 6;       // every amplitude times a complex scalar
    case KOP_DENSE: return 8.0 * (1 << nq) - 2;
    default: return 0;            // exact exchanges
    }
}

LGate lower_gate(int kind, const int *qubits, const double *params, uint64_t gate_id) {
    LGate g;
    g.nq = kind_arity(kind);
    for (int j = 0; j < g.nq; ++j) g.q[j] = qubits[j];
    g.m = kind_matrix(kind, params);
    g.gate_id = gate_id;
    const auto &m = g.m;
    switch (kind) {
    case QTASK_H: case QTASK_RY:  // real matrices
        g.kop = KOP_UR;
        for (int i = 0; i < 4; ++i) g.coef.push_back(m[i].real());
        break;
    case QTASK_RX:  // real diagonal, imaginary off-diagonal
        g.kop = KOP_UX;
        g.coef = {m[0].real(), m[1].imag(), m[2].imag(), m[3].real()};
        break;
    case QTASK_Z: case QTASK_S: case QTASK_SDG: case QTASK_T: case QTASK_TDG:  // diag(1, p)
        g.kop = KOP_P1; g.diagonal = g.monomial = true;
        push(g.coef, m[3]);
        break;
    case QTASK_RZ:
        g.kop = KOP_D1; g.diagonal = g.monomial = true;
        push(g.coef, m[0]); push(g.coef, m[3]);
        break;
    case QTASK_X:
        g.kop = KOP_X1; g.monomial = true;
        break;
    case QTASK_Y:
        g.kop = KOP_A1; g.monomial = true;
        push(g.coef, m[1]); push(g.coef, m[2]);
        break;
    case QTASK_CX:
        g.kop = KOP_CX; g.monomial = true;
        break;
    case QTASK_CZ: case QTASK_CP:  // diag(1, 1, 1, p)
        g.kop = KOP_P2; g.diagonal = g.monomial = true;
        push(g.coef, m[15]);
        break;
    case QTASK_SWAP:
        g.kop = KOP_SWAP; g.monomial = true;
        break;
    case QTASK_CCX:
        g.kop = KOP_CCX; g.monomial = true;
        break;
    default:
        throw std::invalid_argument("gate kind");
    }
    return g;
}

std::vector<cd> embed(const LGate &g, const std::vector<int> &qs) {
    const int k = int(qs.size());
    const int dim = 1 << k;
    const int gd = 1 << g.nq;
    // position of each gate qubit inside qs
    int pos[3];
    uint32_t gmask = 0;
    for (int j = 0; j < g.nq; ++j) {
        pos[j] = -1;
        for (int i = 0; i < k; ++i)
            if (qs[i] == g.q[j]) pos[j] = i;
        if (pos[j] < 0) throw std::logic_error("embed: gate qubit outside the stage");
        gmask |= 1u << pos[j];
    }
    auto local = [&](uint32_t idx) {
        int l = 0;
        for (int j = 0; j < g.nq; ++j) l |= int((idx >> pos[j]) & 1) << (g.nq - 1 - j);
        return l;
    };
    std::vector<cd> u(size_t(dim) * dim, cd(0, 0));
    for (uint32_t r = 0; r < uint32_t(dim); ++r)
        for (uint32_t c = 0; c < uint32_t(dim); ++c)
            if ((r & ~gmask) == (c & ~gmask)) u[size_t(r) * dim + c] = g.m[size_t(local(r)) * gd + local(c)];
    return u;
}

}  // namespace qtask
