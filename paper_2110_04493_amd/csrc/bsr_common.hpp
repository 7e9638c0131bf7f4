// Helpers shared by the 16 x 16 tile kernels (bsr.hip, bsr_adjoint.hip).
//
// Lane layouts of v_mfma_f64_16x16x4f64: A(i, k) comes from lane i + 16k,
// B(k, j) from lane j + 16k, and result (i, j) lands in lane j + 16 (i mod 4),
// register i / 4.  Tiles are stored so that each lane's four operands of a
// 16-deep product are 32 contiguous bytes:
//   A layout: (r, c) at ((c mod 4) 16 + r) 4 + c / 4
//   B layout: (r, c) at ((r mod 4) 16 + c) 4 + r / 4   (= accumulator layout)
// A tile in the A layout is, element for element, its transpose in the B
// layout (and the other way round), so products with T^T need no transposed
// copies.
#pragma once

#include "kernels.hpp"

namespace xpm {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;
constexpr int kTileElems = kTile * kTile;

__device__ __forceinline__ int offA(int r, int c) { return (((c & 3) << 4) + r) * 4 + (c >> 2); }
__device__ __forceinline__ int offB(int r, int c) { return (((r & 3) << 4) + c) * 4 + (r >> 2); }

__device__ __forceinline__ void wfence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Tile index of block column J in block row K, or -1 (rank in the block
// row's bit map).
__device__ __forceinline__ int64_t tile_of(const int32_t *lo, const int64_t *woff, const uint2 *rt,
                                           const int64_t *tb, int64_t K, int J) {
    const int d = J - lo[K];
    const int64_t w0 = woff[K];
    if (d < 0 || (d >> 5) >= woff[K + 1] - w0) return -1;
    const uint2 e = rt[w0 + (d >> 5)];
    const uint32_t bit = 1u << (d & 31);
    if (!(e.x & bit)) return -1;
    return tb[K] + e.y + __popc(e.x & (bit - 1u));
}

// 16-deep product of one A-operand tile with one B-operand tile into acc.
__device__ __forceinline__ d4 mfma16(const d4 &a, const d4 &b, d4 acc) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b[kk], acc, 0, 0, 0);
    return acc;
}

// Lane l's A operand of (2 I_16) for slice kk: 2 where row l % 16 equals
// column 4 kk + l / 16.
__device__ __forceinline__ d4 two_identity_a(int lane) {
    d4 t;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) t[kk] = (lane & 15) == 4 * kk + (lane >> 4) ? 2.0 : 0.0;
    return t;
}

}  // namespace xpm
