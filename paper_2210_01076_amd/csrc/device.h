// Host-side launchers of the HIP kernels (kernels.hip).  All launches are
// asynchronous on `s`; each returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "kdefs.h"

namespace qtask {

// One pass over `n_tiles` tiles of 2^b amplitudes (dtype 0: complex128, 1: complex64).
hipError_t launch_pass(int dtype, const KArgs &a, uint32_t n_tiles, int b, hipStream_t s);

// Whether a pass runs in the matrix-core variant of the pass kernel: it has
// matrix-core stages, or dense stages in complex128 (the complex128
// vector-ALU variant exchanges real and imaginary parts in turn and leaves
// dense stages out).  That variant exchanges whole complex values through
// LDS: 2^b x sizeof(complex) bytes per tile.
inline bool pass_uses_mf(int dtype, const KArgs &a) { return a.has_mfma || (dtype == 0 && a.has_dense); }

// LDS bytes per tile of 2^b amplitudes for a pass kernel variant.
inline uint32_t pass_lds_bytes(int dtype, bool mf, int b) {
    const uint32_t part = dtype == 0 ? 8u : 4u;
    return (1u << b) * (dtype == 0 && !mf ? part : 2u * part);
}

// Batched small-session pass round: the item count is read from `count`
// (device memory); `n_groups` workgroups of `threads` threads and
// `lds_bytes` LDS each (items must all use that thread count).  With `mf`
// set, each item runs in the variant pass_uses_mf picks for it (so the
// result is the one launch_pass gives), and lds_bytes must be
// pass_lds_bytes(dtype, true, b); without it every item must be a pass
// for which pass_uses_mf is false.
hipError_t launch_pass_batch(int dtype, bool mf, const KBatchItem *items, const uint32_t *count, uint32_t n_groups,
                             uint32_t threads, uint32_t lds_bytes, hipStream_t s);
// Batched renormalisation sums (one workgroup per item, count in device memory).
hipError_t launch_batch_sums(const KSumItem *items, const uint32_t *count, uint32_t n_groups, hipStream_t s);

// FP64 sum |a_i|^2 over n elements: partial sums over a fixed grid, then one
// workgroup adds them in a fixed order.  out[0] = sum; when scale_out is not
// null, scale_out[0] = 1/sqrt(sum).
uint32_t reduce_grid(uint64_t n);
hipError_t launch_norm(int dtype, const void *state, uint64_t n, double *partials, double *out,
                       double *scale_out, hipStream_t s);
// Sum of n_partials precomputed partials (fixed order).
hipError_t launch_sum_partials(const double *partials, uint32_t n_partials, double *out, double *scale_out,
                               hipStream_t s);
// <a|b> in FP64: out[0] = re, out[1] = im.  partials needs 2*reduce_grid(n) doubles.
hipError_t launch_inner(int dtype_a, int dtype_b, const void *a, const void *b, uint64_t n, double *partials,
                        double *out, hipStream_t s);
// state *= (R)scale[0]
hipError_t launch_scale(int dtype, void *state, uint64_t n, const double *scale, hipStream_t s);
// Count elements whose bytes differ.  partials needs reduce_grid(n) uint64.
hipError_t launch_compare(int dtype, const void *a, const void *b, uint64_t n, unsigned long long *partials,
                          unsigned long long *out, hipStream_t s);
// Order-independent 64-bit hash of the state bytes.
hipError_t launch_hash(int dtype, const void *a, uint64_t n, unsigned long long *partials,
                       unsigned long long *out, hipStream_t s);
// state = |0...0>
hipError_t launch_fill_basis(int dtype, void *state, uint64_t n, hipStream_t s);
// Block k of the list (2^block_bits elements) from source block src_idx[k]
// to destination block dst_idx[k]; a null index list means k itself; a null
// source fills the destination blocks with their part of |0...0>.
hipError_t launch_block_copy(int dtype, void *dst, const void *src, const uint32_t *dst_idx, const uint32_t *src_idx,
                             uint32_t n_blocks, int block_bits, hipStream_t s);

// Device address (on `device`) and size of the library's fixed scratch
// array for the allocation-free inner product; the address is looked up
// once per device and cached.
hipError_t noalloc_scratch(int device, double **ptr, size_t *doubles);

// dst = src over n 32-byte words (plain streaming copy)
hipError_t launch_copy(void *dst, const void *src, uint64_t n32, hipStream_t s);

}  // namespace qtask
