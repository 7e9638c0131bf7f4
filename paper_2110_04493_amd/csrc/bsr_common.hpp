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

// a[n - 1] of a small register array without a dynamic index (which would
// move the array to scratch memory); n >= 1.
template <int kN>
__device__ __forceinline__ int last_of(const int (&a)[kN], int n) {
    int v = a[0];
#pragma unroll
    for (int t = 1; t < kN; ++t)
        if (t < n) v = a[t];
    return v;
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

// Accumulates acc[t] += sum over items r = 0 .. nr-1, in order, of
// A(r) * B(r, t), 16 x 16 tile products on the matrix cores.  item(r, K, a)
// gives item r's inner index K and its A-operand tile index a; look(K, ti)
// sets ti[t] to the B-operand tile index for output t, leaving -1 where that
// tile is absent.  The indices of 64 items are looked up at once (one item
// per lane, all loads in flight together); the products then walk the items
// with at least one B tile, reading their indices with readlane, and load the
// operands of the next item before issuing the current item's instructions.
// Absent B tiles load tile 0 of Bb (present whenever a product runs) so that
// every stage issues the same loads.
template <int kGroup, class Item, class Look>
__device__ __forceinline__ void pipe_products(int64_t nr, Item item, Look look,
                                              const double *__restrict__ Ab,
                                              const double *__restrict__ Bb,
                                              d4 (&acc)[kGroup]) {
    const int lane = lane_id();
    for (int64_t c0 = 0; c0 < nr; c0 += kWave) {
        int ti[kGroup];
        int ai = 0;
#pragma unroll
        for (int t = 0; t < kGroup; ++t) ti[t] = -1;
        if (c0 + lane < nr) {
            int K;
            item(c0 + lane, K, ai);
            look(K, ti);
        }
        bool any = false;
#pragma unroll
        for (int t = 0; t < kGroup; ++t) any = any || ti[t] >= 0;
        uint64_t m = __ballot(any);
        if (!m) continue;
        int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        int64_t ta = __builtin_amdgcn_readlane(ai, l);
        d4 a = *(const d4 *)(Ab + ta * kTileElems + 4 * lane);
        int bi[kGroup];
        d4 b[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            bi[t] = __builtin_amdgcn_readlane(ti[t], l);
            const int64_t src = bi[t] >= 0 ? bi[t] : 0;
            b[t] = *(const d4 *)(Bb + src * kTileElems + 4 * lane);
        }
        for (;;) {
            const bool more = m != 0;
            d4 a2 = a, b2[kGroup];
            int bi2[kGroup];
#pragma unroll
            for (int t = 0; t < kGroup; ++t) {
                b2[t] = b[t];
                bi2[t] = -1;
            }
            if (more) {
                l = __ffsll((long long)m) - 1;
                m &= m - 1;
                ta = __builtin_amdgcn_readlane(ai, l);
                a2 = *(const d4 *)(Ab + ta * kTileElems + 4 * lane);
#pragma unroll
                for (int t = 0; t < kGroup; ++t) {
                    bi2[t] = __builtin_amdgcn_readlane(ti[t], l);
                    const int64_t src = bi2[t] >= 0 ? bi2[t] : 0;
                    b2[t] = *(const d4 *)(Bb + src * kTileElems + 4 * lane);
                }
            }
#pragma unroll
            for (int t = 0; t < kGroup; ++t)
                if (bi[t] >= 0) acc[t] = mfma16(a, b[t], acc[t]);
            if (!more) break;
            a = a2;
#pragma unroll
            for (int t = 0; t < kGroup; ++t) {
                b[t] = b2[t];
                bi[t] = bi2[t];
            }
        }
    }
}

// Tile index of block column J in a block row whose origin, bit-map words
// and tile base are already loaded (as tile_of), or -1.
__device__ __forceinline__ int tile_in_row(int loK, int64_t w0, int64_t WK, int64_t tbK,
                                           const uint2 *rt, int J) {
    const int d = J - loK;
    if (d < 0 || (d >> 5) >= WK) return -1;
    const uint2 e = rt[w0 + (d >> 5)];
    const uint32_t bit = 1u << (d & 31);
    if (!(e.x & bit)) return -1;
    return (int)(tbK + e.y + __popc(e.x & (bit - 1u)));
}

}  // namespace xpm
