// HIP kernels for gfx950 (CDNA4): the pass kernel that applies a planned
// group of gates to every tile of the state, and the FP64 reductions.
//
// Pass kernel (one workgroup per tile of 2^b amplitudes, 2^(b-4) threads):
//  1. load: each thread reads 16 amplitudes; consecutive lanes read
//     consecutive addresses inside the tile's 2^c-amplitude chunks, so every
//     wave issues fully used 16-byte-per-lane loads;
//  2. the tile goes to LDS at swizzled slots (XOR of the low bits with a
//     linear function of the high bits, so the strided register gathers of
//     the stages below hit distinct banks);
//  3. each stage gathers 16 amplitudes per thread spanning 4 tile qubits,
//     runs its ops on registers (exact exchanges for X/CX/SWAP/CCX, phase
//     scalings for diagonal gates, 2x2/4x4/16x16 complex matrices otherwise)
//     and scatters them back;
//  4. store, optionally also to a checkpoint buffer, optionally only the
//     blocks of an affected-block mask, optionally accumulating the FP64
//     squared norm of the tile.
// All arithmetic is in the state's precision (FP64 for complex128, FP32 for
// complex64); there are no atomics, so every result is a pure function of
// the input and the plan.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.h"

namespace qtask {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

#define NR QK_NREG

// ------------------------------------------------------------ register ops
// Every op updates its registers in place: the products that need an old
// value are formed before the fused multiply-add that overwrites it, so the
// register allocator can keep each amplitude in one register across the op
// loop (no copies at the join of the op switch).  The two amplitudes of a
// pair are updated by the same expression shape, out = fma(diag, own,
// offdiag * other), whichever of them is the 0-side of the qubit.

// fused multiply-add in the state's precision
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// (xr, xi) <- m * (xr, xi) for complex m (a phase or diagonal entry)
template <typename R>
__device__ __forceinline__ void cmul_in_place(R &xr, R &xi, R mr, R mi) {
    const R t = mi * xi, u = mi * xr;
    xr = fmaR(mr, xr, -t);
    xi = fmaR(mr, xi, u);
}

// x <- a x + b y, y <- d y + c x for complex a b c d
template <typename R>
__device__ __forceinline__ void pair_u(R &xr, R &xi, R &yr, R &yi, R ar, R ai, R br, R bi, R cr, R ci, R dr,
                                       R di) {
    const R pr = fmaR(br, yr, -(bi * yi)), pi = fmaR(br, yi, bi * yr);  // b y
    const R qr = fmaR(cr, xr, -(ci * xi)), qi = fmaR(cr, xi, ci * xr);  // c x
    const R sx = fmaR(-ai, xi, pr), tx = fmaR(ai, xr, pi);
    xr = fmaR(ar, xr, sx);
    xi = fmaR(ar, xi, tx);
    const R sy = fmaR(-di, yi, qr), ty = fmaR(di, yr, qi);
    yr = fmaR(dr, yr, sy);
    yi = fmaR(dr, yi, ty);
}

template <int A, typename R>
__device__ __forceinline__ void op_u1(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R m00r = c[0], m00i = c[1], m01r = c[2], m01i = c[3];
    const R m10r = c[4], m10i = c[5], m11r = c[6], m11i = c[7];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << A)) continue;
        const int j = i | (1 << A);
        pair_u(a[i].x, a[i].y, a[j].x, a[j].y, m00r, m00i, m01r, m01i, m10r, m10i, m11r, m11i);
    }
}

template <int A, typename R>
__device__ __forceinline__ void op_d1(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R d0r = c[0], d0i = c[1], d1r = c[2], d1i = c[3];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << A)) cmul_in_place(a[i].x, a[i].y, d1r, d1i);
        else cmul_in_place(a[i].x, a[i].y, d0r, d0i);
    }
}

// Exchange two registers in place (v_swap_b32 on each 32-bit half): the
// values keep their registers, so the op switch joins without copies.
__device__ __forceinline__ void xchg(float &a, float &b) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void xchg(double &a, double &b) {
    uint32_t al = __builtin_bit_cast(uint2, a).x, ah = __builtin_bit_cast(uint2, a).y;
    uint32_t bl = __builtin_bit_cast(uint2, b).x, bh = __builtin_bit_cast(uint2, b).y;
    asm volatile("v_swap_b32 %0, %1" : "+v"(al), "+v"(bl));
    asm volatile("v_swap_b32 %0, %1" : "+v"(ah), "+v"(bh));
    a = __builtin_bit_cast(double, make_uint2(al, ah));
    b = __builtin_bit_cast(double, make_uint2(bl, bh));
}

template <typename R>
__device__ __forceinline__ void swap_amp(typename V2<R>::T (&a)[NR], int i, int j) {
    xchg(a[i].x, a[j].x);
    xchg(a[i].y, a[j].y);
}

template <int A, typename R>
__device__ __forceinline__ void op_a1(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R ar = c[0], ai = c[1], br = c[2], bi = c[3];  // m01, m10
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << A)) continue;
        const int j = i | (1 << A);
        xchg(a[i].x, a[j].x);
        xchg(a[i].y, a[j].y);
        cmul_in_place(a[i].x, a[i].y, ar, ai);
        cmul_in_place(a[j].x, a[j].y, br, bi);
    }
}

template <int A, typename R>
__device__ __forceinline__ void op_x1(typename V2<R>::T (&a)[NR], const R *__restrict__) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if (!(i & (1 << A))) swap_amp<R>(a, i, i | (1 << A));
}

template <int A, int B, typename R>
__device__ __forceinline__ void op_cx(typename V2<R>::T (&a)[NR], const R *__restrict__) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if ((i & (1 << A)) && !(i & (1 << B))) swap_amp<R>(a, i, i | (1 << B));
}

template <int A, int B, typename R>
__device__ __forceinline__ void op_swap(typename V2<R>::T (&a)[NR], const R *__restrict__) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if ((i & (1 << A)) && !(i & (1 << B))) swap_amp<R>(a, i, (i & ~(1 << A)) | (1 << B));
}

template <int A, int B, int C, typename R>
__device__ __forceinline__ void op_ccx(typename V2<R>::T (&a)[NR], const R *__restrict__) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if ((i & (1 << A)) && (i & (1 << B)) && !(i & (1 << C))) swap_amp<R>(a, i, i | (1 << C));
}

template <typename R>
__device__ __forceinline__ void op_dense(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    R xr[NR], xi[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) { xr[i] = a[i].x; xi[i] = a[i].y; }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        R sr = c[2 * NR * r] * xr[0], si = c[2 * NR * r] * xi[0];
        sr = fmaR(-c[2 * NR * r + 1], xi[0], sr);
        si = fmaR(c[2 * NR * r + 1], xr[0], si);
#pragma unroll
        for (int l = 1; l < NR; ++l) {
            const R mr = c[2 * (NR * r + l)], mi = c[2 * (NR * r + l) + 1];
            sr = fmaR(mr, xr[l], sr);
            sr = fmaR(-mi, xi[l], sr);
            si = fmaR(mr, xi[l], si);
            si = fmaR(mi, xr[l], si);
        }
        a[r].x = sr;
        a[r].y = si;
    }
}

template <int A, typename R>
__device__ __forceinline__ void op_ur(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R m00 = c[0], m01 = c[1], m10 = c[2], m11 = c[3];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << A)) continue;
        const int j = i | (1 << A);
        const R pr = m01 * a[j].x, qr = m10 * a[i].x;
        a[i].x = fmaR(m00, a[i].x, pr);
        a[j].x = fmaR(m11, a[j].x, qr);
        const R pi = m01 * a[j].y, qi = m10 * a[i].y;
        a[i].y = fmaR(m00, a[i].y, pi);
        a[j].y = fmaR(m11, a[j].y, qi);
    }
}

// [[a, i b], [i c, d]], a b c d real
template <int A, typename R>
__device__ __forceinline__ void op_ux(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R ca = c[0], b = c[1], cc = c[2], d = c[3];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << A)) continue;
        const int j = i | (1 << A);
        const R p1 = b * a[j].y, p2 = b * a[j].x, q1 = cc * a[i].y, q2 = cc * a[i].x;
        a[i].x = fmaR(ca, a[i].x, -p1);
        a[i].y = fmaR(ca, a[i].y, p2);
        a[j].x = fmaR(d, a[j].x, -q1);
        a[j].y = fmaR(d, a[j].y, q2);
    }
}

template <int A, typename R>
__device__ __forceinline__ void op_p1(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R pr = c[0], pi = c[1];
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if (i & (1 << A)) cmul_in_place(a[i].x, a[i].y, pr, pi);
}

template <int A, int B, typename R>
__device__ __forceinline__ void op_p2(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R pr = c[0], pi = c[1];
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if ((i & (1 << A)) && (i & (1 << B))) cmul_in_place(a[i].x, a[i].y, pr, pi);
}

template <typename R>
__device__ __forceinline__ void op_gph(typename V2<R>::T (&a)[NR], const R *__restrict__ c) {
    const R gr = c[0], gi = c[1];
#pragma unroll
    for (int i = 0; i < NR; ++i) cmul_in_place(a[i].x, a[i].y, gr, gi);
}

// Phase gates with a qubit off the stage's registers.  A site is a lane bit
// (a per-lane condition, applied under the lane mask so that lanes where it
// fails keep their bits untouched: a multiply by 1 + 0i could turn a -0 into
// +0) or a bit of the tile origin (the same in every lane: a wave-uniform
// branch skips the op where it fails).
__device__ __forceinline__ bool origin_off(uint32_t s, uint64_t base) {
    return s >= KPC_ORIGIN && s != KPC_NONE && !((base >> (s - KPC_ORIGIN)) & 1u);
}
__device__ __forceinline__ bool lane_on(uint32_t s, uint32_t t) {
    return s < KPC_LANE || s >= KPC_ORIGIN || ((t >> (s - KPC_LANE)) & 1u);
}

// KOP_PC: p on the registers with bit A set, where site b holds.
template <int A, typename R>
__device__ __forceinline__ void op_pc(typename V2<R>::T (&a)[NR], const R *__restrict__ c, uint32_t site, uint32_t t,
                                      uint64_t base) {
    if (origin_off(site, base)) return;
    if (lane_on(site, t)) {
        const R pr = c[0], pi = c[1];
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (i & (1 << A)) cmul_in_place(a[i].x, a[i].y, pr, pi);
    }
}

// The lane's pending phase: phase gates whose qubits are all off the
// registers scale every register of a lane alike, and they commute with
// every register op of the stage, so their product is formed first (one
// complex multiply each) and applied to the registers once, by KOP_PHI.
template <typename R> struct Pending {
    R r, i;
    uint32_t hit;  // 0 or 1 per lane (a lane value, not a lane mask the op loop would carry in scalars)
};

template <typename R>
__device__ __forceinline__ void op_pcl(Pending<R> &ph, const R *__restrict__ c, uint32_t sa, uint32_t sb, uint32_t t,
                                       uint64_t base) {
    if (origin_off(sa, base) || origin_off(sb, base)) return;
    if (lane_on(sa, t) && lane_on(sb, t)) {
        cmul_in_place(ph.r, ph.i, c[0], c[1]);
        ph.hit = 1u;
    }
}

template <typename R>
__device__ __forceinline__ void op_phi(typename V2<R>::T (&a)[NR], Pending<R> &ph) {
    if (ph.hit != 0u) {
        const R pr = ph.r, pi = ph.i;
#pragma unroll
        for (int i = 0; i < NR; ++i) cmul_in_place(a[i].x, a[i].y, pr, pi);
    }
    ph.r = R(1);
    ph.i = R(0);
    ph.hit = 0u;
}

#define SW1(F)                                   \
    switch (op.a) {                              \
    case 0: F<0>(a, c); break;              \
    case 1: F<1>(a, c); break;              \
    case 2: F<2>(a, c); break;              \
    default: F<3>(a, c); break;             \
    }

#define SW2(F)                                   \
    switch (op.a * 4 + op.b) {                   \
    case 1: F<0, 1>(a, c); break;           \
    case 2: F<0, 2>(a, c); break;           \
    case 3: F<0, 3>(a, c); break;           \
    case 4: F<1, 0>(a, c); break;           \
    case 6: F<1, 2>(a, c); break;           \
    case 7: F<1, 3>(a, c); break;           \
    case 8: F<2, 0>(a, c); break;           \
    case 9: F<2, 1>(a, c); break;           \
    case 11: F<2, 3>(a, c); break;          \
    case 12: F<3, 0>(a, c); break;          \
    case 13: F<3, 1>(a, c); break;          \
    case 14: F<3, 2>(a, c); break;          \
    default: break;                              \
    }

// controls a < b, target c
#define SW3(F)                                   \
    switch (op.a * 16 + op.b * 4 + op.c) {       \
    case 0 * 16 + 1 * 4 + 2: F<0, 1, 2>(a, c); break; \
    case 0 * 16 + 1 * 4 + 3: F<0, 1, 3>(a, c); break; \
    case 0 * 16 + 2 * 4 + 1: F<0, 2, 1>(a, c); break; \
    case 0 * 16 + 2 * 4 + 3: F<0, 2, 3>(a, c); break; \
    case 0 * 16 + 3 * 4 + 1: F<0, 3, 1>(a, c); break; \
    case 0 * 16 + 3 * 4 + 2: F<0, 3, 2>(a, c); break; \
    case 1 * 16 + 2 * 4 + 0: F<1, 2, 0>(a, c); break; \
    case 1 * 16 + 2 * 4 + 3: F<1, 2, 3>(a, c); break; \
    case 1 * 16 + 3 * 4 + 0: F<1, 3, 0>(a, c); break; \
    case 1 * 16 + 3 * 4 + 2: F<1, 3, 2>(a, c); break; \
    case 2 * 16 + 3 * 4 + 0: F<2, 3, 0>(a, c); break; \
    case 2 * 16 + 3 * 4 + 1: F<2, 3, 1>(a, c); break; \
    default: break;                              \
    }

#define SW1PC(F)                                           \
    switch (op.a) {                                        \
    case 0: F<0, R>(a, c, op.b, t, base); break;           \
    case 1: F<1, R>(a, c, op.b, t, base); break;           \
    case 2: F<2, R>(a, c, op.b, t, base); break;           \
    default: F<3, R>(a, c, op.b, t, base); break;          \
    }

// DN: the variant runs dense 16x16 register ops (the complex128 vector-ALU
// kernel leaves them to the matrix-core variant: their 32 extra registers
// would cost it a wave per SIMD)
template <typename R, bool DN>
__device__ __forceinline__ void apply_op(const KOp op, typename V2<R>::T (&a)[NR], const R *__restrict__ c, uint32_t t,
                                         uint64_t base, Pending<R> &ph) {
    // the rotations and the CX of layered circuits first: a wave-uniform
    // if-chain reaches them in one or two branches
    const uint32_t ty = op.type;
    if (ty == KOP_UR) { SW1(op_ur) }
    else if (ty == KOP_UX) { SW1(op_ux) }
    else if (ty == KOP_D1) { SW1(op_d1) }
    else if (ty == KOP_CX) { SW2(op_cx) }
    else {
        switch (ty) {
        case KOP_U1: SW1(op_u1) break;
        case KOP_A1: SW1(op_a1) break;
        case KOP_X1: SW1(op_x1) break;
        case KOP_SWAP: SW2(op_swap) break;
        case KOP_CCX: SW3(op_ccx) break;
        case KOP_DENSE:
            if constexpr (DN) op_dense(a, c);
            break;
        case KOP_P1: SW1(op_p1) break;
        case KOP_P2: SW2(op_p2) break;
        case KOP_GPH: op_gph<R>(a, c); break;
        case KOP_PC: SW1PC(op_pc) break;
        case KOP_PCL: op_pcl<R>(ph, c, op.a, op.b, t, base); break;
        case KOP_PHI: op_phi<R>(a, ph); break;
        default: break;
        }
    }
}

// ----------------------------------------------------- barriers, reduce
// Workgroup barrier that orders LDS only.  The pass kernels never read global
// memory written by another thread of the same launch, so the barrier does
// not need to drain outstanding global loads (which would cancel the
// prefetch of the next tile).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over the workgroup in a fixed order: a butterfly inside each wave,
// then wave results added in wave order by thread 0.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = v;
    lds_barrier();
    double s = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += scratch[w];
    }
    return s;  // valid in thread 0
}

// ------------------------------------------------------------- pass body
// The leading fields of a stage record, read with one wide scalar load.
struct StageHead {
    uint32_t reg_bit[QK_G];
    uint32_t thr_off[QK_MAX_THR_BITS];
    uint32_t op_begin, op_count;
    uint32_t kind;
};
static_assert(sizeof(StageHead) == 64, "stage head is one 64-byte scalar load");
static_assert(offsetof(KStage, thr_off) == offsetof(StageHead, thr_off) &&
                  offsetof(KStage, op_begin) == offsetof(StageHead, op_begin) &&
                  offsetof(KStage, kind) == offsetof(StageHead, kind),
              "stage head mirrors the start of KStage");

__device__ __forceinline__ StageHead stage_head(const KStage *__restrict__ S) {
    return *reinterpret_cast<const StageHead *>(S);
}

// Runs the stage's ops.  `op` holds the stage's first record on entry and the
// record after its last one on exit: consecutive stages have consecutive op
// ranges, so it is the next stage's first record.  Each record is loaded
// before the previous op runs (the op array is followed by a spare record
// inside the plan blob, so the read past the last op stays in bounds).
template <typename R, bool DN>
__device__ __forceinline__ void run_ops(const StageHead &h, const KOp *__restrict__ ops, const R *__restrict__ coefs,
                                        typename V2<R>::T (&a)[NR], KOp &op, uint32_t t, uint64_t base,
                                        Pending<R> &ph) {
    const uint32_t oe = h.op_begin + h.op_count;
    for (uint32_t oi = h.op_begin; oi < oe; ++oi) {
        const KOp nx = ops[oi + 1];
        apply_op<R, DN>(op, a, coefs + op.coef, t, base, ph);
        op = nx;
    }
}

// The loops run over the table's full length with branch-free selects: the
// table is read by a few wide scalar loads, with one wait, and no lane
// diverges.  Entries past the stage's thread bits are zero and so are the
// corresponding bits of t (t < 2^n_thr), so they add nothing.
__device__ __forceinline__ uint32_t thr_lds(const StageHead &h, uint32_t t) {
    uint32_t o = 0;
#pragma unroll
    for (int k = 0; k < QK_MAX_THR_BITS; ++k) o ^= h.thr_off[k] & (0u - ((t >> k) & 1u));
    return o;
}

// Per-register LDS slots (XOR) and global offsets (OR) from the per-bit
// contributions; each register adds one bit to an earlier one.
__device__ __forceinline__ void reg_slots(const StageHead &h, uint32_t bt, uint32_t (&sl)[NR]) {
    const uint32_t b0 = h.reg_bit[0], b1 = h.reg_bit[1], b2 = h.reg_bit[2], b3 = h.reg_bit[3];
    sl[0] = bt;
#pragma unroll
    for (int i = 1; i < NR; ++i) {
        const int low = i & -i;
        const uint32_t bb = low == 1 ? b0 : low == 2 ? b1 : low == 4 ? b2 : b3;
        sl[i] = sl[i & (i - 1)] ^ bb;
    }
}

__device__ __forceinline__ void reg_goffs(const KStage *__restrict__ S, uint64_t g0, uint64_t (&g)[NR]) {
    const uint64_t b0 = S->g_bit[0], b1 = S->g_bit[1], b2 = S->g_bit[2], b3 = S->g_bit[3];
    g[0] = g0;
#pragma unroll
    for (int i = 1; i < NR; ++i) {
        const int low = i & -i;
        const uint64_t bb = low == 1 ? b0 : low == 2 ? b1 : low == 4 ? b2 : b3;
        g[i] = g[i & (i - 1)] | bb;
    }
}

__device__ __forceinline__ uint64_t thr_glb(const KStage *__restrict__ S, uint32_t t) {
    uint64_t o = 0;
#pragma unroll
    for (int k = 0; k < QK_MAX_THR_BITS; ++k) o |= S->g_thr[k] & (uint64_t(0) - ((t >> k) & 1u));
    return o;
}

// ------------------------------------------------------------ MFMA stage
// Y = U X for one dense 2^K x 2^K complex unitary on the stage's K tile bits,
// over all 2^(b-K) columns of the tile held in LDS.  The complex product is
// done as the real block product [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Xr; Xi]
// (no 3-multiplication trick, so rounding matches a plain complex product)
// with 16x16x4 MFMA tiles: each wave owns 2^(6-K) column blocks of 16 columns
// and all 2^(K-3) row blocks, reads its columns, accumulates, then writes the
// same columns back (waves never touch each other's columns).
template <typename R> struct MfmaT;
template <> struct MfmaT<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output register i of lane l holds row 4*i + l/16 of the 16x16 block
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct MfmaT<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output register i of lane l holds row 4*(l/16) + i of the 16x16 block
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// N consecutive values from p with vector loads of up to 16 bytes (p is
// aligned to the load size).
template <typename R, int N>
__device__ __forceinline__ void load_vec(const R *__restrict__ p, R (&v)[N]) {
    constexpr int W = N * int(sizeof(R)) >= 16 ? 16 / int(sizeof(R)) : N;
    typedef R vt __attribute__((ext_vector_type(W)));
#pragma unroll
    for (int c = 0; c < N / W; ++c) {
        const vt w = reinterpret_cast<const vt *>(p)[c];
#pragma unroll
        for (int j = 0; j < W; ++j) v[c * W + j] = w[j];
    }
}

template <typename R, int K>
__device__ __forceinline__ void mfma_stage_k(const KStage *__restrict__ S, const R *__restrict__ coefs,
                                             R *__restrict__ lr) {
    using M = MfmaT<R>;
    constexpr int DIM = 1 << K;     // complex dimension
    constexpr int MR = 2 * DIM;     // real rows = real inner dimension
    constexpr int RB = MR / 16;     // row blocks
    constexpr int KS = MR / 4;      // inner steps of 4
    constexpr int CB = 64 / DIM;    // column blocks per wave
    // the whole A operand stays in registers while it fits: 4 * KS * RB
    // bytes per lane (64 VGPRs at K = 5 in FP32, 32 at K = 4 in FP64)
    constexpr bool A_REG = sizeof(R) == 4 ? K <= 5 : K <= 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the planner stores the block operand in lane order: this lane's RB
    // values of step s (rows 16 rb + lane % 16, column 4 s + lane / 16) are
    // contiguous at (s * 64 + lane) * RB
    const R *__restrict__ A = coefs + S->coef + lane * RB;
    // LDS slot contributions (the slot map is linear over the bits of the
    // row and column indices): unrolled branch-free selects over the tables,
    // whose unused entries are zero
    uint32_t lane_off = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) lane_off ^= S->col_off[j] & (0u - ((uint32_t(lane) >> j) & 1u));
    uint32_t cb_off[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const uint32_t blk = uint32_t(wave * CB + cb);
        uint32_t o = lane_off;
#pragma unroll
        for (int j = 4; j < QK_MAX_TILE_BITS; ++j) o ^= S->col_off[j] & (0u - ((blk >> (j - 4)) & 1u));
        cb_off[cb] = o;
    }
    uint32_t rbit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) rbit[j] = S->row_off[1 << j];
    auto row_slot = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) o ^= rbit[j] & (0u - ((uint32_t(r) >> j) & 1u));
        return o;
    };
    R areg[A_REG ? KS : 1][RB];
    if constexpr (A_REG) {
#pragma unroll
        for (int s = 0; s < KS; ++s) load_vec<R, RB>(A + s * 64 * RB, areg[s]);
    }
    typename M::acc_t acc[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = typename M::acc_t{0, 0, 0, 0};
    auto step = [&](int s, const R (&av)[RB]) {
        const int kk = 4 * s + (lane >> 4);          // real inner index of this lane
        const uint32_t roff = row_slot(kk & (DIM - 1));
        const int part = kk >= DIM ? 1 : 0;          // 0: Xr, 1: Xi
        R bv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) bv[cb] = lr[2 * (cb_off[cb] ^ roff) + part];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = M::mma(av[rb], bv[cb], acc[rb][cb]);
    };
    if constexpr (A_REG) {
#pragma unroll
        for (int s = 0; s < KS; ++s) step(s, areg[s]);
    } else {
#pragma unroll 4
        for (int s = 0; s < KS; ++s) {
            R av[RB];
            load_vec<R, RB>(A + s * 64 * RB, av);
            step(s, av);
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 16 * rb + M::row(lane, i);
            const uint32_t roff = row_slot(rr & (DIM - 1));
            const int part = rr >= DIM ? 1 : 0;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) lr[2 * (cb_off[cb] ^ roff) + part] = acc[rb][cb][i];
        }
}

template <typename R>
__device__ __forceinline__ void mfma_stage(const KStage *__restrict__ S, const R *__restrict__ coefs,
                                           typename V2<R>::T *__restrict__ lds) {
    R *lr = reinterpret_cast<R *>(lds);
    switch (S->k) {
    case 4: mfma_stage_k<R, 4>(S, coefs, lr); break;
    case 5: mfma_stage_k<R, 5>(S, coefs, lr); break;
    case 6: mfma_stage_k<R, 6>(S, coefs, lr); break;
    default: break;
    }
}

// Deposit runs of a pass, read once into scalar registers (a fixed-size
// unrolled copy keeps them out of memory inside the tile loop).
struct TileRuns {
    uint32_t n;
    uint32_t run[QK_MAX_RUNS];
};

__device__ __forceinline__ TileRuns load_runs(const KPass *__restrict__ P) {
    TileRuns tr;
    tr.n = P->n_runs;
#pragma unroll
    for (int r = 0; r < QK_MAX_RUNS; ++r) tr.run[r] = P->run[r];
    return tr;
}

// Global offset of tile `tile`: its index bits deposited at the non-tile
// qubits, one run of consecutive qubits at a time.
__device__ __forceinline__ uint64_t tile_origin(const TileRuns &tr, uint32_t tile) {
    uint64_t base = 0;
#pragma unroll
    for (int r = 0; r < QK_MAX_RUNS; ++r) {
        if (r < int(tr.n)) {
            const uint32_t src = tr.run[r] & 0xffu, len = (tr.run[r] >> 8) & 0xffu, dst = tr.run[r] >> 16;
            base |= uint64_t((tile >> src) & ((1u << len) - 1u)) << dst;
        }
    }
    return base;
}

// Whether the kernel exchanges a tile between stages as real parts, then
// imaginary parts, through an LDS area of 2^b values instead of 2^b complex
// values (the complex128 vector-ALU kernel: its LDS per tile halves, so more
// workgroups fit on a CU).
template <typename R, bool MF> constexpr bool split_lds() { return sizeof(R) == 8 && !MF; }

// Whether a pass kernel variant runs dense 16x16 register ops (KOP_DENSE);
// passes with such ops go to the matrix-core variant in complex128.
template <typename R, bool MF> constexpr bool dense_ops() { return MF || sizeof(R) == 4; }

// One tile (number idx of the pass, or tile_list[idx]).  The first stage's
// registers come straight from global memory, the middle stages go through
// LDS, the last stage's registers go straight back to global memory.
template <typename R, bool MF>
__device__ __forceinline__ void pass_tile(uint32_t idx, const uint32_t *__restrict__ tile_list, void *dst_,
                                          const void *src_, void *ckpt_, const KPass *__restrict__ P,
                                          const KStage *__restrict__ stages, const KOp *__restrict__ ops,
                                          const R *__restrict__ coefs, const uint64_t *__restrict__ store_mask,
                                          const double *__restrict__ scale, double *__restrict__ partials,
                                          uint32_t src_basis, uint32_t block_bits,
                                          typename V2<R>::T *__restrict__ lds) {
    using C = typename V2<R>::T;
    const uint32_t t = threadIdx.x;
    const uint32_t n_thr = P->n_thr;
    const uint32_t ns = P->stage_count;
    const KStage *__restrict__ S0 = stages + P->stage_begin;
    const KStage *__restrict__ SL = S0 + (ns - 1);
    const uint32_t tile = tile_list ? tile_list[idx] : idx;
    const uint64_t base = tile_origin(load_runs(P), tile);

    // One loop over the stages with a single op-loop site: stage 0 gathers
    // from global memory, the others from LDS; every stage but the last
    // scatters back to LDS.  (One call site keeps the amplitude registers
    // in place across the whole pass.)
    constexpr bool SPLIT = split_lds<R, MF>();
    C a[NR];
    Pending<R> ph{R(1), R(0), 0u};
    KOp op = ops[S0->op_begin];
    for (uint32_t si = 0; si < ns; ++si) {
        const KStage *__restrict__ S = S0 + si;
        const StageHead h = stage_head(S);
        if (MF && h.kind == KSTAGE_MFMA) {
            mfma_stage<R>(S, coefs, lds);
            lds_barrier();
            continue;
        }
        uint32_t bt = thr_lds(h, t);
        uint32_t sl[NR];
        reg_slots(h, bt, sl);
        if (si == 0) {
            uint64_t g[NR];
            reg_goffs(S, base | thr_glb(S, t), g);
            if (src_basis) {
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    a[i].x = g[i] == 0 ? R(1) : R(0);
                    a[i].y = R(0);
                }
            } else {
                const C *src = static_cast<const C *>(src_);
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const C y = src[g[i]];
                    a[i].x = y.x;
                    a[i].y = y.y;
                }
                if (scale) {
                    const R sc = R(scale[0]);
#pragma unroll
                    for (int i = 0; i < NR; ++i) { a[i].x *= sc; a[i].y *= sc; }
                }
            }
        } else if (!SPLIT) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const C y = lds[sl[i]];
                a[i].x = y.x;
                a[i].y = y.y;
            }
        }
        run_ops<R, dense_ops<R, MF>()>(h, ops, coefs, a, op, t, base, ph);
        if (si + 1 == ns) break;
        if constexpr (SPLIT) {
            // real parts, then imaginary parts, through half the LDS: each
            // thread writes its slots of this stage and reads its slots of
            // the next; the barrier between a read and the next write keeps
            // a slot from being overwritten before its reader has it
            asm volatile("" : "+v"(bt));
            reg_slots(h, bt, sl);
            const StageHead h2 = stage_head(S + 1);
            uint32_t sl2[NR];
            reg_slots(h2, thr_lds(h2, t), sl2);
            R *lr = reinterpret_cast<R *>(lds);
#pragma unroll
            for (int i = 0; i < NR; ++i) lr[sl[i]] = a[i].x;
            lds_barrier();
#pragma unroll
            for (int i = 0; i < NR; ++i) a[i].x = lr[sl2[i]];
            lds_barrier();
#pragma unroll
            for (int i = 0; i < NR; ++i) lr[sl[i]] = a[i].y;
            lds_barrier();
#pragma unroll
            for (int i = 0; i < NR; ++i) a[i].y = lr[sl2[i]];
            continue;
        }
        // complex128: recompute the slots instead of keeping them live across
        // the op loop (16 fewer registers; see the kernel's occupancy hint)
        if constexpr (sizeof(R) == 8) {
            asm volatile("" : "+v"(bt));
            reg_slots(h, bt, sl);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            C y;
            y.x = a[i].x;
            y.y = a[i].y;
            lds[sl[i]] = y;
        }
        lds_barrier();
    }

    // store: plain (the common case), or only the blocks of the mask, and
    // optionally the tile's squared norm; each option is a wave-uniform branch
    C *dst = static_cast<C *>(dst_);
    C *ck = static_cast<C *>(ckpt_);
    uint64_t g[NR];
    reg_goffs(SL, base | thr_glb(SL, t), g);
    if (!store_mask) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            C y;
            y.x = a[i].x;
            y.y = a[i].y;
            dst[g[i]] = y;
        }
        if (ck) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                C y;
                y.x = a[i].x;
                y.y = a[i].y;
                ck[g[i]] = y;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            C y;
            y.x = a[i].x;
            y.y = a[i].y;
            const uint64_t blk = g[i] >> block_bits;
            if ((store_mask[blk >> 6] >> (blk & 63)) & 1) {
                dst[g[i]] = y;
                if (ck) ck[g[i]] = y;
            }
        }
    }
    if (partials) {
        double acc = 0;
#pragma unroll
        for (int i = 0; i < NR; ++i) acc += double(a[i].x) * double(a[i].x) + double(a[i].y) * double(a[i].y);
        __shared__ double red[16];
        const double sum = block_sum(acc, red);
        if (threadIdx.x == 0) partials[idx] = sum;
    }
}

// Pass kernel: one workgroup per tile.
template <typename R, bool MF>
__global__ void __launch_bounds__(512)
qk_pass(void *dst, const void *src, void *ckpt, const KPass *__restrict__ pass, const KStage *__restrict__ stages,
        const KOp *__restrict__ ops, const R *__restrict__ coefs, const uint32_t *__restrict__ tile_list,
        const uint64_t *__restrict__ store_mask, const double *__restrict__ scale, double *__restrict__ partials,
        uint32_t src_basis, uint32_t block_bits) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = typename V2<R>::T;
    pass_tile<R, MF>(blockIdx.x, tile_list, dst, src, ckpt, pass, stages, ops, coefs, store_mask, scale, partials,
                     src_basis, block_bits, reinterpret_cast<C *>(smem));
}

// The complex128 vector-ALU kernel asks for four waves per SIMD (128
// registers; a few values of the tile setup then live in scratch, outside
// the op loop), which its half-size LDS exchange leaves room for.  The
// matrix-core variants would spill under the same limit and keep the
// default.
template <>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
qk_pass<double, false>(void *dst, const void *src, void *ckpt, const KPass *__restrict__ pass,
                       const KStage *__restrict__ stages, const KOp *__restrict__ ops,
                       const double *__restrict__ coefs, const uint32_t *__restrict__ tile_list,
                       const uint64_t *__restrict__ store_mask, const double *__restrict__ scale,
                       double *__restrict__ partials, uint32_t src_basis, uint32_t block_bits) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass_tile<double, false>(blockIdx.x, tile_list, dst, src, ckpt, pass, stages, ops, coefs, store_mask, scale,
                             partials, src_basis, block_bits, reinterpret_cast<V2<double>::T *>(smem));
}

// Batched pass round over many small sessions that share one tile shape.
// The item table and its length live in device memory, so a captured graph
// of such launches can be replayed with new work each time.  Each workgroup
// finds its item by binary search over the items' first workgroup index;
// every decision below depends only on blockIdx and the table, so a
// workgroup either runs the whole pass body or leaves before any barrier.
// The MF instantiation holds both pass bodies and runs, per item, the one
// the single-session launcher would pick (matrix-core stages, or dense
// stages in complex128, take the matrix-core body), so a session's result
// does not depend on which sessions share its round.
template <typename R, bool MF>
__global__ void __launch_bounds__(512)
qk_pass_batch(const KBatchItem *__restrict__ items, const uint32_t *__restrict__ count) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = typename V2<R>::T;
    const uint32_t n_items = count[0];
    if (n_items == 0) return;
    uint32_t lo = 0, hi = n_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].tile_begin <= blockIdx.x) lo = mid; else hi = mid;
    }
    const KBatchItem *it = items + lo;
    if (blockIdx.x < it->tile_begin) return;
    const uint32_t local = blockIdx.x - it->tile_begin;
    if (local >= it->n_tiles || it->threads != blockDim.x) return;
    const KArgs &a = it->args;
    if constexpr (MF) {
        if (a.has_mfma || (sizeof(R) == 8 && a.has_dense)) {
            pass_tile<R, true>(local, a.tile_list, a.dst, a.src, a.ckpt, a.pass, a.stages, a.ops,
                               static_cast<const R *>(a.coefs), a.store_mask, a.scale, a.partials, a.src_basis,
                               a.block_bits, reinterpret_cast<C *>(smem));
            return;
        }
    }
    pass_tile<R, false>(local, a.tile_list, a.dst, a.src, a.ckpt, a.pass, a.stages,
                         a.ops, static_cast<const R *>(a.coefs), a.store_mask, a.scale, a.partials, a.src_basis,
                         a.block_bits, reinterpret_cast<C *>(smem));
}

// Batched renormalisation sums: workgroup i adds the per-tile partials of
// item i in a fixed order and writes the norm and 1/sqrt(norm).
__global__ void __launch_bounds__(256)
qk_batch_sums(const KSumItem *__restrict__ items, const uint32_t *__restrict__ count) {
    if (blockIdx.x >= count[0]) return;
    const KSumItem &it = items[blockIdx.x];
    double acc = 0;
    for (uint32_t i = threadIdx.x; i < it.n; i += 256) acc += it.partials[i];
    __shared__ double red[4];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) {
        it.norm_out[0] = tot;
        it.scale_out[0] = 1.0 / sqrt(tot);
    }
}

// ------------------------------------------------------------- reductions
constexpr int RED_THREADS = 256;

uint32_t reduce_grid(uint64_t n) {
    const uint64_t per = uint64_t(RED_THREADS) * 16;
    uint64_t g = (n + per - 1) / per;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return uint32_t(g);
}

template <typename R>
__global__ void __launch_bounds__(RED_THREADS) qk_norm_partials(const void *state_, uint64_t n, double *partials) {
    using C = typename V2<R>::T;
    const C *s = static_cast<const C *>(state_);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t beg = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += RED_THREADS) {
        const C x = s[i];
        acc += double(x.x) * double(x.x) + double(x.y) * double(x.y);
    }
    __shared__ double red[RED_THREADS / 64];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename RA, typename RB>
__global__ void __launch_bounds__(RED_THREADS)
qk_inner_partials(const void *a_, const void *b_, uint64_t n, double *partials) {
    using CA = typename V2<RA>::T;
    using CB = typename V2<RB>::T;
    const CA *a = static_cast<const CA *>(a_);
    const CB *b = static_cast<const CB *>(b_);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t beg = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    double re = 0, im = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += RED_THREADS) {
        const CA x = a[i];
        const CB y = b[i];
        const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
        re += xr * yr + xi * yi;
        im += xr * yi - xi * yr;
    }
    __shared__ double red[RED_THREADS / 64];
    const double tr = block_sum(re, red);
    lds_barrier();
    const double ti = block_sum(im, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = tr;
        partials[2 * blockIdx.x + 1] = ti;
    }
}

// One workgroup adds `n` partials (stride `stride`, offset `off`) in a fixed order.
__global__ void __launch_bounds__(RED_THREADS)
qk_sum_partials(const double *partials, uint32_t n, uint32_t stride, double *out, double *scale_out) {
    double acc = 0;
    for (uint32_t i = threadIdx.x; i < n; i += RED_THREADS) acc += partials[size_t(i) * stride];
    __shared__ double red[RED_THREADS / 64];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) {
        out[0] = tot;
        if (scale_out) scale_out[0] = 1.0 / sqrt(tot);
    }
}

template <typename R>
__global__ void qk_scale(void *state_, uint64_t n, const double *scale) {
    using C = typename V2<R>::T;
    C *s = static_cast<C *>(state_);
    const R sc = R(scale[0]);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        C x = s[i];
        x.x *= sc;
        x.y *= sc;
        s[i] = x;
    }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    // splitmix64 finaliser (Steele, Lea, Flood: "Fast splittable pseudorandom number generators")
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long *scratch) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < int((blockDim.x + 63) >> 6); ++w) s += scratch[w];
    return s;
}

// Elements are compared / hashed as raw words: W = 2 (complex128) or 1
// (complex64) 64-bit words per element.
template <int W>
__global__ void __launch_bounds__(RED_THREADS)
qk_compare(const unsigned long long *a, const unsigned long long *b, uint64_t n, unsigned long long *partials) {
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t beg = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    unsigned long long cnt = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += RED_THREADS) {
        bool diff = false;
#pragma unroll
        for (int w = 0; w < W; ++w) diff |= a[W * i + w] != b[W * i + w];
        cnt += diff ? 1 : 0;
    }
    __shared__ unsigned long long red[RED_THREADS / 64];
    const unsigned long long tot = block_sum_u64(cnt, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <int W>
__global__ void __launch_bounds__(RED_THREADS)
qk_hash(const unsigned long long *a, uint64_t n, unsigned long long *partials) {
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t beg = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    unsigned long long h = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += RED_THREADS) {
#pragma unroll
        for (int w = 0; w < W; ++w) h += mix64(a[W * i + w] ^ mix64((W * i + w) * 0x9e3779b97f4a7c15ull + 1));
    }
    __shared__ unsigned long long red[RED_THREADS / 64];
    const unsigned long long tot = block_sum_u64(h, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void qk_sum_u64(const unsigned long long *partials, uint32_t n, unsigned long long *out) {
    unsigned long long acc = 0;
    for (uint32_t i = threadIdx.x; i < n; i += RED_THREADS) acc += partials[i];
    __shared__ unsigned long long red[RED_THREADS / 64];
    const unsigned long long tot = block_sum_u64(acc, red);
    if (threadIdx.x == 0) out[0] = tot;
}

template <typename R>
__global__ void qk_fill_basis(void *state_, uint64_t n) {
    using C = typename V2<R>::T;
    C *s = static_cast<C *>(state_);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        C x;
        x.x = i == 0 ? R(1) : R(0);
        x.y = R(0);
        s[i] = x;
    }
}

// Whole blocks of 2^block_bits amplitudes: block k of the list goes from
// source block src_idx[k] to destination block dst_idx[k] (a missing index
// list means the block number k itself).  Without a source the destination
// blocks get the matching part of |0...0>.  Used to capture and restore
// sparse checkpoints (only the blocks a segment can change).
template <typename R>
__global__ void qk_block_copy(void *dst_, const void *src_, const uint32_t *dst_idx, const uint32_t *src_idx,
                              uint32_t n_blocks, int block_bits) {
    using C = typename V2<R>::T;
    C *dst = static_cast<C *>(dst_);
    const C *src = static_cast<const C *>(src_);
    const uint64_t bsz = uint64_t(1) << block_bits;
    for (uint32_t bi = blockIdx.x; bi < n_blocks; bi += gridDim.x) {
        const uint64_t d = uint64_t(dst_idx ? dst_idx[bi] : bi) << block_bits;
        if (src) {
            const uint64_t so = uint64_t(src_idx ? src_idx[bi] : bi) << block_bits;
            for (uint64_t i = threadIdx.x; i < bsz; i += blockDim.x) dst[d + i] = src[so + i];
        } else {
            for (uint64_t i = threadIdx.x; i < bsz; i += blockDim.x) {
                C z;
                z.x = d + i == 0 ? R(1) : R(0);
                z.y = R(0);
                dst[d + i] = z;
            }
        }
    }
}

// Plain streaming copy: each thread moves one 16-byte word with non-temporal
// accesses, one short-lived workgroup per 4 KiB (the form that reaches the
// highest copy rate on the device; a grid-stride loop over fewer workgroups
// and unrolled variants measured 15-25 % lower).
typedef double qk_nd2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(256) qk_copy(qk_nd2 *__restrict__ dst, const qk_nd2 *__restrict__ src, uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---------------------------------------------------------------- launchers
namespace {
// Workgroups above 64 KiB of dynamic LDS need an explicit opt-in per kernel.
hipError_t allow_lds(const void *fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

uint32_t fill_grid(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    return uint32_t(g < 1 ? 1 : g);
}
}  // namespace

template <typename R, bool MF>
hipError_t launch_pass_t(const KArgs &a, uint32_t n_tiles, int b, hipStream_t s) {
    static_assert(split_lds<R, MF>() == (sizeof(R) == 8 && !MF), "pass_lds_bytes assumes this exchange rule");
    const uint32_t threads = 1u << (b - QK_G);
    const size_t lds = pass_lds_bytes(sizeof(R) == 8 ? 0 : 1, MF, b);
    hipError_t e = allow_lds(reinterpret_cast<const void *>(&qk_pass<R, MF>), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((qk_pass<R, MF>), dim3(n_tiles), dim3(threads), lds, s, a.dst, a.src, a.ckpt, a.pass,
                       a.stages, a.ops, static_cast<const R *>(a.coefs), a.tile_list, a.store_mask, a.scale,
                       a.partials, a.src_basis, a.block_bits);
    return hipGetLastError();
}

hipError_t launch_pass(int dtype, const KArgs &a, uint32_t n_tiles, int b, hipStream_t s) {
    (void)hipGetLastError();  // start from a clean error state
    if (n_tiles == 0) return hipSuccess;
    if (pass_uses_mf(dtype, a))
        return dtype == 0 ? launch_pass_t<double, true>(a, n_tiles, b, s) : launch_pass_t<float, true>(a, n_tiles, b, s);
    return dtype == 0 ? launch_pass_t<double, false>(a, n_tiles, b, s) : launch_pass_t<float, false>(a, n_tiles, b, s);
}

template <typename R, bool MF>
hipError_t launch_pass_batch_t(const KBatchItem *items, const uint32_t *count, uint32_t n_groups, uint32_t threads,
                               uint32_t lds_bytes, hipStream_t s) {
    hipError_t e = allow_lds(reinterpret_cast<const void *>(&qk_pass_batch<R, MF>), lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((qk_pass_batch<R, MF>), dim3(n_groups), dim3(threads), lds_bytes, s, items, count);
    return hipGetLastError();
}

hipError_t launch_pass_batch(int dtype, bool mf, const KBatchItem *items, const uint32_t *count, uint32_t n_groups,
                             uint32_t threads, uint32_t lds_bytes, hipStream_t s) {
    (void)hipGetLastError();
    if (dtype == 0)
        return mf ? launch_pass_batch_t<double, true>(items, count, n_groups, threads, lds_bytes, s)
                  : launch_pass_batch_t<double, false>(items, count, n_groups, threads, lds_bytes, s);
    return mf ? launch_pass_batch_t<float, true>(items, count, n_groups, threads, lds_bytes, s)
              : launch_pass_batch_t<float, false>(items, count, n_groups, threads, lds_bytes, s);
}

hipError_t launch_batch_sums(const KSumItem *items, const uint32_t *count, uint32_t n_groups, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(qk_batch_sums, dim3(n_groups), dim3(256), 0, s, items, count);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, uint32_t n_partials, double *out, double *scale_out,
                               hipStream_t s) {
    hipLaunchKernelGGL(qk_sum_partials, dim3(1), dim3(RED_THREADS), 0, s, partials, n_partials, 1u, out, scale_out);
    return hipGetLastError();
}

hipError_t launch_norm(int dtype, const void *state, uint64_t n, double *partials, double *out, double *scale_out,
                       hipStream_t s) {
    const uint32_t g = reduce_grid(n);
    if (dtype == 0)
        hipLaunchKernelGGL(qk_norm_partials<double>, dim3(g), dim3(RED_THREADS), 0, s, state, n, partials);
    else
        hipLaunchKernelGGL(qk_norm_partials<float>, dim3(g), dim3(RED_THREADS), 0, s, state, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(partials, g, out, scale_out, s);
}

hipError_t launch_inner(int dtype_a, int dtype_b, const void *a, const void *b, uint64_t n, double *partials,
                        double *out, hipStream_t s) {
    const uint32_t g = reduce_grid(n);
    (void)hipGetLastError();
    if (dtype_a == 0 && dtype_b == 0)
        hipLaunchKernelGGL((qk_inner_partials<double, double>), dim3(g), dim3(RED_THREADS), 0, s, a, b, n, partials);
    else if (dtype_a == 0)
        hipLaunchKernelGGL((qk_inner_partials<double, float>), dim3(g), dim3(RED_THREADS), 0, s, a, b, n, partials);
    else if (dtype_b == 0)
        hipLaunchKernelGGL((qk_inner_partials<float, double>), dim3(g), dim3(RED_THREADS), 0, s, a, b, n, partials);
    else
        hipLaunchKernelGGL((qk_inner_partials<float, float>), dim3(g), dim3(RED_THREADS), 0, s, a, b, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qk_sum_partials, dim3(1), dim3(RED_THREADS), 0, s, partials, g, 2u, out, (double *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qk_sum_partials, dim3(1), dim3(RED_THREADS), 0, s, partials + 1, g, 2u, out + 1,
                       (double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_scale(int dtype, void *state, uint64_t n, const double *scale, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(qk_scale<double>, dim3(fill_grid(n)), dim3(256), 0, s, state, n, scale);
    else
        hipLaunchKernelGGL(qk_scale<float>, dim3(fill_grid(n)), dim3(256), 0, s, state, n, scale);
    return hipGetLastError();
}

hipError_t launch_compare(int dtype, const void *a, const void *b, uint64_t n, unsigned long long *partials,
                          unsigned long long *out, hipStream_t s) {
    const uint32_t g = reduce_grid(n);
    const auto *pa = static_cast<const unsigned long long *>(a);
    const auto *pb = static_cast<const unsigned long long *>(b);
    if (dtype == 0)
        hipLaunchKernelGGL(qk_compare<2>, dim3(g), dim3(RED_THREADS), 0, s, pa, pb, n, partials);
    else
        hipLaunchKernelGGL(qk_compare<1>, dim3(g), dim3(RED_THREADS), 0, s, pa, pb, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qk_sum_u64, dim3(1), dim3(RED_THREADS), 0, s, partials, g, out);
    return hipGetLastError();
}

hipError_t launch_hash(int dtype, const void *a, uint64_t n, unsigned long long *partials, unsigned long long *out,
                       hipStream_t s) {
    const uint32_t g = reduce_grid(n);
    const auto *pa = static_cast<const unsigned long long *>(a);
    if (dtype == 0)
        hipLaunchKernelGGL(qk_hash<2>, dim3(g), dim3(RED_THREADS), 0, s, pa, n, partials);
    else
        hipLaunchKernelGGL(qk_hash<1>, dim3(g), dim3(RED_THREADS), 0, s, pa, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qk_sum_u64, dim3(1), dim3(RED_THREADS), 0, s, partials, g, out);
    return hipGetLastError();
}

hipError_t launch_fill_basis(int dtype, void *state, uint64_t n, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(qk_fill_basis<double>, dim3(fill_grid(n)), dim3(256), 0, s, state, n);
    else
        hipLaunchKernelGGL(qk_fill_basis<float>, dim3(fill_grid(n)), dim3(256), 0, s, state, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, uint64_t n32, hipStream_t s) {
    (void)hipGetLastError();
    const uint64_t n16 = 2 * n32;
    const uint64_t g = (n16 + 255) / 256;
    if (g > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(qk_copy, dim3(uint32_t(g < 1 ? 1 : g)), dim3(256), 0, s, static_cast<qk_nd2 *>(dst),
                       static_cast<const qk_nd2 *>(src), n16);
    return hipGetLastError();
}

hipError_t launch_block_copy(int dtype, void *dst, const void *src, const uint32_t *dst_idx, const uint32_t *src_idx,
                             uint32_t n_blocks, int block_bits, hipStream_t s) {
    (void)hipGetLastError();
    if (n_blocks == 0) return hipSuccess;
    const uint32_t g = n_blocks < 65535 ? n_blocks : 65535;
    if (dtype == 0)
        hipLaunchKernelGGL(qk_block_copy<double>, dim3(g), dim3(256), 0, s, dst, src, dst_idx, src_idx, n_blocks,
                           block_bits);
    else
        hipLaunchKernelGGL(qk_block_copy<float>, dim3(g), dim3(256), 0, s, dst, src, dst_idx, src_idx, n_blocks,
                           block_bits);
    return hipGetLastError();
}

// --------------------------------------------- allocation-free scratch
// Partial sums for the allocation-free inner product: a fixed device array
// (one copy per GPU, held until the process ends), big enough for the
// largest reduction grid (2 * reduce_grid(n) partials plus the two results).
// Host code never passes the array's name to a kernel: that is a host-side
// stand-in, not a device address.  The device address is taken once per
// device with hipGetSymbolAddress, with that device current, and kept.
constexpr size_t kNoallocScratchDoubles = 2 * 2048 + 2;
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {nullptr};
}  // namespace

hipError_t noalloc_scratch(int device, double **ptr, size_t *doubles) {
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[device];
    *doubles = kNoallocScratchDoubles;
    return hipSuccess;
}

}  // namespace qtask
