// Adjoint squaring step on 16 x 16 tiles (gfx950 FP64 matrix cores).
//
// For the squarings of Eq. (4.15) with frozen masks, the gradient moves back
// one step as  G_{k-1} = P_{k-1}(2 G_k + G_k T^T + T^T G_k),  T = T_{k-1},
// where P_{k-1} keeps the stored entries of T_{k-1}.  On tiles, for every
// tile (I, J) of T's pattern:
//   2 G_IJ                = (2 I_16) G_IJ                 (G_IJ, B layout)
//   (G T^T)_IJ = sum_K G_IK (T_JK)^T                      (G_IK A layout, T_JK A layout
//                                                          read as the B operand)
//   (T^T G)_IJ = sum_K (T_KI)^T G_KJ                      (T_KI B layout read as the
//                                                          A operand, G_KJ B layout)
// then the mask keeps the slots where T_IJ is nonzero.  The K sums run over
// G's block row I and over T's block column I (T^T's block row I, kept as a
// sorted list), in ascending K, so the result is bitwise reproducible.
#include "bsr_common.hpp"

namespace xpm {

constexpr int kAdjGroup = 4;      // output tiles per wave (work item)
constexpr bool kAdjSplit = true;  // the step as two kernels (see k_bsr_adjoint)

// ----------------------------------------------------------------- T^T's block rows

__global__ void k_bsr_colcount(int64_t nb, const int32_t *lo, const int64_t *woff,
                               const uint2 *rt, int64_t *cnt) {
    const int64_t K = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (K >= nb) return;
    for (int64_t w = woff[K] + lane_id(); w < woff[K + 1]; w += kWave) {
        uint32_t x = rt[w].x;
        const int base = lo[K] + 32 * (int)(w - woff[K]);
        while (x) {
            const int J = base + __ffs(x) - 1;
            x &= x - 1;
            atomicAdd((unsigned long long *)&cnt[J], 1ull);
        }
    }
}

__global__ void k_bsr_colfill(int64_t nb, const int32_t *lo, const int64_t *woff,
                              const uint2 *rt, const int64_t *tb, int64_t *fill, int32_t *uk,
                              int64_t *ut) {
    const int64_t K = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (K >= nb) return;
    for (int64_t w = woff[K] + lane_id(); w < woff[K + 1]; w += kWave) {
        const uint2 e = rt[w];
        uint32_t x = e.x;
        unsigned r = e.y;
        const int base = lo[K] + 32 * (int)(w - woff[K]);
        while (x) {
            const int J = base + __ffs(x) - 1;
            x &= x - 1;
            const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&fill[J], 1ull);
            uk[pos] = (int32_t)K;
            ut[pos] = tb[K] + r;
            ++r;
        }
    }
}

// Sorts each block column's list by K (ranks are distinct: one tile per
// (K, J)), from the unsorted (uk, ut) into (ck, ct).
__global__ void k_bsr_colsort(const int64_t *ptr, int64_t nb, const int32_t *uk, const int64_t *ut,
                              int32_t *ck, int64_t *ct) {
    const int64_t J = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (J >= nb) return;
    const int64_t b = ptr[J], e = ptr[J + 1];
    for (int64_t p = b + lane_id(); p < e; p += kWave) {
        const int32_t k = uk[p];
        int64_t r = 0;
        for (int64_t q = b; q < e; ++q) r += uk[q] < k;
        ck[b + r] = k;
        ct[b + r] = ut[p];
    }
}

// ----------------------------------------------------------------- adjoint tiles

// One wave per work item: a block row I of T and up to kGroup of its tiles.
// kPart 0 computes the whole step; kPart 1 only 2 G + G T^T (unmasked, into
// out) and kPart 2 adds T^T G to it, masks, and writes both layouts: the two
// halves need fewer registers each, so more waves fit on a SIMD.  kSym: T is
// symmetric and assembled in the B layout only (tA unused).
template <int kGroup, int kPart, bool kSym>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_bsr_adjoint(
    int64_t nb,
    // T = T_{k-1}: pattern (with each tile's block column) and tiles
    const int32_t *__restrict__ tlo, const int64_t *__restrict__ twoff,
    const uint2 *__restrict__ trt, const int64_t *__restrict__ ttb,
    const int32_t *__restrict__ tcols, const double *__restrict__ tA,
    const double *__restrict__ tB,
    // G on T_k's pattern
    const int32_t *__restrict__ glo, const int64_t *__restrict__ gwoff,
    const uint2 *__restrict__ grt, const int64_t *__restrict__ gtb,
    const int32_t *__restrict__ gcols, const double *__restrict__ gA,
    const double *__restrict__ gB,
    // T's block columns (T^T's block rows), sorted by K
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ ck,
    const int64_t *__restrict__ ct,
    const int64_t *__restrict__ gofs, const int32_t *__restrict__ owner,
    double *__restrict__ out, double *__restrict__ outA, const int64_t *__restrict__ nwork_dev,
    int xcd) {
    const int lane = lane_id();
    // blocks of four work items; with xcd, contiguous ranges of blocks per
    // XCD (the grid covers a bound of the count, plus 8 blocks)
    const int64_t nw = *nwork_dev, wpb = blockDim.x / kWave;
    const int64_t blk = xcd ? xcd_item(blockIdx.x, (nw + wpb - 1) / wpb) : (int64_t)blockIdx.x;
    if (blk < 0) return;
    const int64_t w = blk * wpb + threadIdx.x / kWave;
    if (w >= nw) return;
    const int64_t I = owner[w];   // the block row: gofs[I] <= w < gofs[I + 1]
    const int64_t t0 = (w - gofs[I]) * kGroup;             // first tile (rank in block row I)
    const int64_t cntI = ttb[I + 1] - ttb[I];
    const int ng = (int)min<int64_t>(kGroup, cntI - t0);
    // block columns J of the group: tiles t0 .. t0 + ng - 1 of T's block row I
    // (past ng, a valid block index that is never used)
    int J[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) J[t] = t < ng ? tcols[ttb[I] + t0 + t] : (int)I;
    d4 acc[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    if constexpr (kPart == 2) {
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            if (t >= ng) break;
            acc[t] = *(const d4 *)(out + (ttb[I] + t0 + t) * kTileElems + 4 * lane);
        }
    }
    if constexpr (kPart != 2) {
        const d4 two = two_identity_a(lane);
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            if (t >= ng) break;
            const int64_t tg = tile_of(glo, gwoff, grt, gtb, I, J[t]);
            if (tg >= 0)
                acc[t] = mfma16(two, *(const d4 *)(gB + tg * kTileElems + 4 * lane), acc[t]);
        }
    }
    // (G T^T)_IJ = sum over K in G's block row I of G_IK (T_JK)^T
    if constexpr (kPart != 2) {
        int loJ[kGroup], tbJ[kGroup];
        int64_t w0J[kGroup], WJ[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            const int Jt = J[t];
            loJ[t] = tlo[Jt];
            w0J[t] = twoff[Jt];
            WJ[t] = t < ng ? twoff[Jt + 1] - w0J[t] : 0;
            tbJ[t] = (int)ttb[Jt];
        }
        const int64_t g0 = gtb[I];
        auto item = [&](int64_t r, int &K, int &a) {
            K = gcols[g0 + r];
            a = (int)(g0 + r);
        };
        if constexpr (kSym) {
            // (T_JK)^T = T_KJ: tile J of T's block row K, in the B layout
            const int jlo = J[0], jhi = last_of(J, ng);
            auto look = [&](int K, int (&ti)[kGroup]) {
                const int loK = tlo[K];
                const int64_t w0 = twoff[K], WK = twoff[K + 1] - w0;
                if (WK == 0 || jhi < loK || jlo >= loK + 32 * (int)WK) return;
                const int64_t tbK = ttb[K];
#pragma unroll
                for (int t = 0; t < kGroup; ++t)
                    if (t < ng) ti[t] = tile_in_row(loK, w0, WK, tbK, trt, J[t]);
            };
            pipe_products<kGroup>(gtb[I + 1] - g0, item, look, gA, tB, acc);
        } else {
            // tile K of T's block row J in the A layout, read as a B
            // operand, is (T_JK)^T
            auto look = [&](int K, int (&ti)[kGroup]) {
#pragma unroll
                for (int t = 0; t < kGroup; ++t)
                    ti[t] = tile_in_row(loJ[t], w0J[t], WJ[t], tbJ[t], trt, K);
            };
            pipe_products<kGroup>(gtb[I + 1] - g0, item, look, gA, tA, acc);
        }
    }
    if constexpr (kPart == 1) {
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            if (t >= ng) break;
            *(d4 *)(out + (ttb[I] + t0 + t) * kTileElems + 4 * lane) = acc[t];
        }
        return;
    }
    // (T^T G)_IJ = sum over K in T's block column I of (T_KI)^T G_KJ
    {
        const int64_t p0 = cptr[I];
        const int jlo = J[0], jhi = last_of(J, ng);
        auto item = [&](int64_t r, int &K, int &a) {
            K = ck[p0 + r];
            a = (int)ct[p0 + r];
        };
        auto look = [&](int K, int (&ti)[kGroup]) {
            const int loK = glo[K];
            const int64_t w0 = gwoff[K], WK = gwoff[K + 1] - w0;
            if (WK == 0 || jhi < loK || jlo >= loK + 32 * (int)WK) return;
            const int64_t tbK = gtb[K];
#pragma unroll
            for (int t = 0; t < kGroup; ++t)
                if (t < ng) ti[t] = tile_in_row(loK, w0, WK, tbK, grt, J[t]);
        };
        pipe_products<kGroup>(cptr[I + 1] - p0, item, look, tB, gB, acc);
    }
    // mask by T's stored entries (T_IJ in the B layout = accumulator layout)
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        if (t >= ng) break;
        const int64_t tt = ttb[I] + t0 + t;
        const d4 m = *(const d4 *)(tB + tt * kTileElems + 4 * lane);
        d4 o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = m[r] != 0.0 ? acc[t][r] : 0.0;
        // the new gradient's tiles are read only by the next adjoint step:
        // streaming stores keep them from displacing this step's operands
        __builtin_nontemporal_store(o, (d4 *)(out + tt * kTileElems + 4 * lane));
        if (!outA) continue;
        // the same tile in the A operand layout: o[r] is entry (4 r + lane / 16,
        // lane % 16)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            __builtin_nontemporal_store(o[r],
                                        &outA[tt * kTileElems + offA(4 * r + (lane >> 4), lane & 15)]);
    }
}

// Values of the output tiles at T's stored entries (CSR order).
__global__ void k_bsr_gather(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                             const int64_t *tb, const double *tiles, double *out) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= T.n) return;
    const int64_t I = i >> 4;
    const int r = (int)(i & 15);
    for (int64_t p = T.rp[i] + lane_id(); p < T.rp[i + 1]; p += kWave) {
        const int j = T.ci[p];
        const int64_t t = tile_of(lo, woff, rt, tb, I, j >> 4);
        out[p] = tiles[t * kTileElems + offB(r, j & 15)];
    }
}

// Work items of four tiles per block row, from the tile bases tb.
__global__ void k_bsr_groups4(const int64_t *tb, int64_t nb, int64_t *gcnt) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nb) gcnt[I] = (tb[I + 1] - tb[I] + kAdjGroup - 1) / kAdjGroup;
}

// ----------------------------------------------------------------- wrappers

hipError_t bsr_groups4(const int64_t *tb, int64_t nb, int64_t *gcnt, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_groups4, dim3((nb + 255) / 256), dim3(256), 0, st, tb, nb, gcnt);
    return hipGetLastError();
}

hipError_t bsr_colcount(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                        int64_t *cnt, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_colcount, dim3((nb + 3) / 4), dim3(256), 0, st, nb, lo, woff, rt,
                       cnt);
    return hipGetLastError();
}

hipError_t bsr_colfill(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                       const int64_t *tb, int64_t *fill, int32_t *uk, int64_t *ut,
                       hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_colfill, dim3((nb + 3) / 4), dim3(256), 0, st, nb, lo, woff, rt, tb,
                       fill, uk, ut);
    return hipGetLastError();
}

hipError_t bsr_colsort(const int64_t *ptr, int64_t nb, const int32_t *uk, const int64_t *ut,
                       int32_t *ck, int64_t *ct, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_colsort, dim3((nb + 3) / 4), dim3(256), 0, st, ptr, nb, uk, ut, ck,
                       ct);
    return hipGetLastError();
}

hipError_t bsr_adjoint(int64_t nb, const int32_t *tlo, const int64_t *twoff, const uint2 *trt,
                       const int64_t *ttb, const int32_t *tcols, const double *tA,
                       const double *tB, const int32_t *glo,
                       const int64_t *gwoff, const uint2 *grt, const int64_t *gtb,
                       const int32_t *gcols, const double *gA, const double *gB,
                       const int64_t *cptr, const int32_t *ck, const int64_t *ct,
                       const int64_t *gofs, const int32_t *owner, double *out, double *outA,
                       const int64_t *nwork_dev, int64_t nwork, hipStream_t st, bool symT) {
    if (nwork == 0) return hipSuccess;
    static const int xcd = [] {
        const char *e = getenv("EXPM_TILE_XCD");
        return e && e[0] == '0' ? 0 : 1;
    }();
    const dim3 grid((unsigned)((nwork + 3) / 4 + 8)), block(256);
#define XPM_ADJ_ARGS                                                                           \
    nb, tlo, twoff, trt, ttb, tcols, tA, tB, glo, gwoff, grt, gtb, gcols, gA, gB, cptr, ck, ct, \
        gofs, owner, out, outA, nwork_dev, xcd
    if (symT) {
        hipLaunchKernelGGL((k_bsr_adjoint<kAdjGroup, 1, true>), grid, block, 0, st, XPM_ADJ_ARGS);
        hipLaunchKernelGGL((k_bsr_adjoint<kAdjGroup, 2, true>), grid, block, 0, st, XPM_ADJ_ARGS);
    } else if (kAdjSplit) {
        hipLaunchKernelGGL((k_bsr_adjoint<kAdjGroup, 1, false>), grid, block, 0, st, XPM_ADJ_ARGS);
        hipLaunchKernelGGL((k_bsr_adjoint<kAdjGroup, 2, false>), grid, block, 0, st, XPM_ADJ_ARGS);
    } else {
        hipLaunchKernelGGL((k_bsr_adjoint<kAdjGroup, 0, false>), grid, block, 0, st, XPM_ADJ_ARGS);
    }
#undef XPM_ADJ_ARGS
    return hipGetLastError();
}

hipError_t bsr_gather(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                      const int64_t *tb, const double *tiles, double *out, hipStream_t st) {
    if (T.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_gather, dim3((T.n + 3) / 4), dim3(256), 0, st, T, lo, woff, rt, tb,
                       tiles, out);
    return hipGetLastError();
}

}  // namespace xpm
