/*
 * CPU oracle for the incremental state-vector path.  TEST INFRASTRUCTURE
 * ONLY: nothing in the product library links, loads or calls this file; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * What it computes (paper, Section II-A "Quantum Circuits and Simulation"):
 * a state of n qubits is 2^n complex amplitudes alpha_b, index b = sum_k q_k 2^k
 * (the last qubit is the most significant bit, Section III-B).  A net (level)
 * acts as the Kronecker product of its gates' matrices padded with identities,
 * and the circuit is the ordered product of the nets.  Applying that product
 * to a vector is the same as applying each gate's small matrix to every group
 * of amplitudes that differ only in the gate's qubits, which is what this file
 * does, one gate at a time, with no blocking, fusion or reordering.
 *
 * Conventions where the paper is silent (each is listed in the design notes):
 *  - gate matrices: X, H and CX exactly as printed in Section II-A; CX has
 *    its control on the high bit of the 2-qubit local index, so for a gate
 *    listed with qubits (q0, q1, ...) the local index is
 *    bit(q0) * 2^(k-1) + ... + bit(q_{k-1}) (first-listed qubit = high bit);
 *  - Y = [[0,-i],[i,0]], Z = diag(1,-1), S = diag(1,i) (square root of Z,
 *    Table I), T = diag(1,e^{i pi/4}) (square root of S, Table I), SDG and
 *    TDG their conjugates;
 *  - RX/RY/RZ(theta) = exp(-i theta P / 2) for P = X, Y, Z;
 *  - CZ = diag(1,1,1,-1), SWAP exchanges |01> and |10>,
 *    CP(lambda) = diag(1,1,1,e^{i lambda}), CCX flips the target when both
 *    controls are 1.
 *
 * Floating point: complex128 as explicit (re, im) double pairs, built with
 * -ffp-contract=off, so each complex multiply-add is four products and
 * rounded sums in a fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Oracle-private gate codes (the Python wrapper maps names to these). */
enum {
    OK_H = 0, OK_X, OK_Y, OK_Z, OK_S, OK_SDG, OK_T, OK_TDG,
    OK_RX, OK_RY, OK_RZ, OK_CX, OK_CZ, OK_SWAP, OK_CP, OK_CCX, OK_COUNT
};

static int arity(int kind)
{
    if (kind >= OK_H && kind <= OK_RZ) return 1;
    if (kind >= OK_CX && kind <= OK_CP) return 2;
    if (kind == OK_CCX) return 3;
    return -1;
}

int oracle_gate_arity(int kind) { return arity(kind); }

/* Fill m (row-major, interleaved re/im, dim x dim with dim = 2^arity) with the
 * gate's matrix.  Returns the dimension, or -1 for an unknown kind. */
int oracle_gate_matrix(int kind, const double *params, double *m)
{
    const int k = arity(kind);
    if (k < 0) return -1;
    const int dim = 1 << k;
    memset(m, 0, sizeof(double) * 2 * dim * dim);
#define SET(r, c, re, im) do { m[2 * ((r) * dim + (c))] = (re); m[2 * ((r) * dim + (c)) + 1] = (im); } while (0)
    const double h = 1.0 / sqrt(2.0);
    double th, cs, sn;
    switch (kind) {
    case OK_H: SET(0, 0, h, 0); SET(0, 1, h, 0); SET(1, 0, h, 0); SET(1, 1, -h, 0); break;
    case OK_X: SET(0, 1, 1, 0); SET(1, 0, 1, 0); break;
    case OK_Y: SET(0, 1, 0, -1); SET(1, 0, 0, 1); break;
    case OK_Z: SET(0, 0, 1, 0); SET(1, 1, -1, 0); break;
    case OK_S: SET(0, 0, 1, 0); SET(1, 1, 0, 1); break;
    case OK_SDG: SET(0, 0, 1, 0); SET(1, 1, 0, -1); break;
    case OK_T: SET(0, 0, 1, 0); SET(1, 1, h, h); break;
    case OK_TDG: SET(0, 0, 1, 0); SET(1, 1, h, -h); break;
    case OK_RX:
        th = params[0] / 2; cs = cos(th); sn = sin(th);
        SET(0, 0, cs, 0); SET(0, 1, 0, -sn); SET(1, 0, 0, -sn); SET(1, 1, cs, 0); break;
    case OK_RY:
        th = params[0] / 2; cs = cos(th); sn = sin(th);
        SET(0, 0, cs, 0); SET(0, 1, -sn, 0); SET(1, 0, sn, 0); SET(1, 1, cs, 0); break;
    case OK_RZ:
        th = params[0] / 2; cs = cos(th); sn = sin(th);
        SET(0, 0, cs, -sn); SET(1, 1, cs, sn); break;
    case OK_CX: SET(0, 0, 1, 0); SET(1, 1, 1, 0); SET(2, 3, 1, 0); SET(3, 2, 1, 0); break;
    case OK_CZ: SET(0, 0, 1, 0); SET(1, 1, 1, 0); SET(2, 2, 1, 0); SET(3, 3, -1, 0); break;
    case OK_SWAP: SET(0, 0, 1, 0); SET(1, 2, 1, 0); SET(2, 1, 1, 0); SET(3, 3, 1, 0); break;
    case OK_CP:
        SET(0, 0, 1, 0); SET(1, 1, 1, 0); SET(2, 2, 1, 0);
        SET(3, 3, cos(params[0]), sin(params[0])); break;
    case OK_CCX:
        for (int i = 0; i < 6; ++i) SET(i, i, 1, 0);
        SET(6, 7, 1, 0); SET(7, 6, 1, 0); break;
    default: return -1;
    }
#undef SET
    return dim;
}

/* Apply one k-qubit matrix m to psi (2^n interleaved complex doubles). */
static void apply_gate(int n, double *psi, int k, const int *q, const double *m, int nthreads)
{
    const int64_t N = (int64_t)1 << n;
    const int dim = 1 << k;
    uint64_t mask = 0;
    for (int j = 0; j < k; ++j) mask |= (uint64_t)1 << q[j];
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t i = 0; i < N; ++i) {
        if ((uint64_t)i & mask) continue; /* one base index per group */
        uint64_t idx[8];
        double in_re[8], in_im[8];
        for (int l = 0; l < dim; ++l) {
            uint64_t g = (uint64_t)i;
            for (int j = 0; j < k; ++j)
                if ((l >> (k - 1 - j)) & 1) g |= (uint64_t)1 << q[j];
            idx[l] = g;
            in_re[l] = psi[2 * g];
            in_im[l] = psi[2 * g + 1];
        }
        for (int r = 0; r < dim; ++r) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < dim; ++c) {
                const double mr = m[2 * (r * dim + c)], mi = m[2 * (r * dim + c) + 1];
                sr += mr * in_re[c] - mi * in_im[c];
                si += mr * in_im[c] + mi * in_re[c];
            }
            psi[2 * idx[r]] = sr;
            psi[2 * idx[r] + 1] = si;
        }
    }
}

/*
 * Apply n_gates gates in order to psi in place.
 *   kinds[g]       oracle gate code
 *   qubits[3*g+j]  j-th listed qubit (controls first), unused slots ignored
 *   params[3*g+j]  angles
 * Returns 0, or -1 on a bad gate (unknown kind, qubit out of range, repeated
 * qubit); psi is left partially updated in that case.
 */
int oracle_apply(int n, double *psi, int n_gates, const int *kinds,
                 const int *qubits, const double *params, int nthreads)
{
    double m[2 * 64];
    for (int g = 0; g < n_gates; ++g) {
        const int k = arity(kinds[g]);
        if (k < 0) return -1;
        const int *q = qubits + 3 * g;
        for (int j = 0; j < k; ++j) {
            if (q[j] < 0 || q[j] >= n) return -1;
            for (int j2 = 0; j2 < j; ++j2)
                if (q[j2] == q[j]) return -1;
        }
        oracle_gate_matrix(kinds[g], params + 3 * g, m);
        apply_gate(n, psi, k, q, m, nthreads);
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
