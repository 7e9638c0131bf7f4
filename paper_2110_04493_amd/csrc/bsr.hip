// Squaring product on 16 x 16 dense tiles with FP64 matrix cores (gfx950).
//
// Once the filtered iterate's band has filled in, T_{i-1} is held as
// block-sparse rows of dense 16 x 16 tiles and T~ = 2T + T*T is formed tile by
// tile with v_mfma_f64_16x16x4f64: C_IJ = (2 I) T_IJ + sum_K T_IK T_KJ, four
// matrix instructions per tile product.  The candidate stays in tile form for
// the filter (Algorithm 4.1 runs on the flat tile values; padding and
// structural zeros add nothing to any sum), and the compaction writes the kept
// entries straight back to CSR.
//
// Lane layouts of v_mfma_f64_16x16x4f64 (one double per lane for A and B,
// four for the accumulator): A(i, k) comes from lane i + 16k, B(k, j) from
// lane j + 16k, and the result (i, j) lands in lane j + 16 (i mod 4), register
// i / 4.  Tiles are stored so that each lane's four operands of a 16-deep
// product are 32 contiguous bytes:
//   A layout: (r, c) at ((c mod 4) 16 + r) 4 + c / 4
//   B layout: (r, c) at ((r mod 4) 16 + c) 4 + r / 4   (= accumulator layout)
//
// Block rows carry a bit map of their block columns (origin a multiple of
// 32 block columns) with prefix counts, so the tile of block column J is
// found in O(1) by rank, as in the scalar product.
#include <stdlib.h>

#include "bsr_common.hpp"

namespace xpm {

constexpr int kPanel = 4;        // block rows per panel (one wave each)
constexpr int kPanelGroup = 2;   // output tiles per wave

// ----------------------------------------------------------------- T -> tiles

// Per block row: origin (block column, multiple of 32) and bit-map words.
__global__ void k_bsr_bounds(CsrView T, int64_t nb, int32_t *lo, int64_t *words) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= nb) return;
    const int64_t r0 = I * kTile, r1 = min<int64_t>(r0 + kTile, T.n);
    // one lane per row of the block row
    int mn = INT32_MAX, mx = -1;
    const int64_t i = r0 + lane_id();
    if (lane_id() < kTile && i < r1) {
        const int64_t b = T.rp[i], e = T.rp[i + 1];
        if (e > b) {
            mn = T.ci[b] >> 4;
            mx = T.ci[e - 1] >> 4;
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane_id() == 0) {
        if (mx < 0) {
            lo[I] = 0;
            words[I] = 0;
        } else {
            const int l = mn & ~31;
            lo[I] = l;
            words[I] = ((mx - l) >> 5) + 1;
        }
    }
}

// Bit map of the block columns of each block row, as (word, prefix) pairs,
// and the tile count.  The bit map is built in LDS (at most n / 512 words).
__global__ __launch_bounds__(64) void k_bsr_bitmap(CsrView T, int64_t nb, const int32_t *lo,
                                                   const int64_t *woff, uint2 *rt, int64_t *cnt) {
    extern __shared__ uint32_t bm[];
    const int64_t I = blockIdx.x;
    if (I >= nb) return;
    const int lane = lane_id();
    const int64_t w0 = woff[I], W = woff[I + 1] - w0;
    if (W == 0) {
        if (lane == 0) cnt[I] = 0;
        return;
    }
    for (int64_t w = lane; w < W; w += kWave) bm[w] = 0;
    wfence();
    const int base = lo[I];
    // the block row's 16 rows are one contiguous range of entries; four
    // chunks of 64 are loaded before their bits are set.  Within a row the
    // columns ascend, so neighbouring lanes mostly share a block column:
    // only the first lane of each run sets its bit (a dense row would
    // otherwise send 64 atomics per instruction to the same word)
    const int64_t p0 = T.rp[I * kTile], p1 = T.rp[min<int64_t>(I * kTile + kTile, T.n)];
    for (int64_t q = p0; q < p1; q += 4 * kWave) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = q + u * kWave + lane;
            c[u] = p < p1 ? T.ci[p] >> 4 : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int prev = __shfl_up(c[u], 1);
            if (c[u] >= 0 && (lane == 0 || prev != c[u])) {
                const int d = c[u] - base;
                atomicOr(&bm[d >> 5], 1u << (d & 31));
            }
        }
    }
    wfence();
    unsigned carry = 0;
    for (int64_t b0 = 0; b0 < W; b0 += kWave) {
        const int64_t w = b0 + lane;
        const uint32_t x = w < W ? bm[w] : 0u;
        const unsigned pc = __popc(x);
        const unsigned inc = wave_incl_scan(pc);
        if (w < W) rt[w0 + w] = make_uint2(x, carry + inc - pc);
        carry += __shfl(inc, kWave - 1);
    }
    if (lane == 0) cnt[I] = carry;
}

// Block column and block row of every tile, in tile order (block rows in
// order, columns ascending within a block row).
__global__ void k_bsr_tcols(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                            const int64_t *tb, int32_t *tcols, int32_t *trows) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= nb) return;
    const int64_t w0 = woff[I], W = woff[I + 1] - w0;
    for (int64_t w = lane_id(); w < W; w += kWave) {
        const uint2 e = rt[w0 + w];
        uint32_t x = e.x;
        int64_t q = tb[I] + e.y;
        while (x) {
            trows[q] = (int32_t)I;
            tcols[q++] = lo[I] + 32 * (int)w + __ffs(x) - 1;
            x &= x - 1;
        }
    }
}

// Row segments: for every tile and each of its 16 rows, the first CSR entry
// of that row inside the tile and the entry count, packed as
// (position << 5) | count (0 for none; the table starts zeroed).
__global__ void k_bsr_seg(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                          const int64_t *tb, int64_t *seg) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= T.n) return;
    const int64_t I = i >> 4;
    const int r = (int)(i & 15);
    const int lane = lane_id();
    const int64_t b = T.rp[i], e = T.rp[i + 1];
    const int loI = lo[I];
    const int64_t w0 = woff[I], tbI = tb[I];
    const unsigned long long above = lane == kWave - 1 ? 0ull : ~0ull << (lane + 1);
    // chunks of 64 entries; the next chunk's block columns are loaded while
    // the current one is handled, and they also give the length of the
    // chunk's last segment (a segment holds at most 16 entries, so it ends
    // within the next chunk)
    int J = b + lane < e ? T.ci[b + lane] >> 4 : INT32_MAX;
    int Jprev = -1;   // block column of the previous chunk's last entry
    for (int64_t c0 = b; c0 < e; c0 += kWave) {
        const int64_t p = c0 + lane, pn = p + kWave;
        const bool valid = p < e;
        const int d = J - loI;
        uint2 w = make_uint2(0u, 0u);
        if (valid) w = rt[w0 + (d >> 5)];
        const int Jn = pn < e ? T.ci[pn] >> 4 : INT32_MAX;
        const int Jlast = __builtin_amdgcn_readlane(J, kWave - 1);
        const unsigned long long cont = __ballot(pn < e && Jn == Jlast);
        int Jp = __shfl_up(J, 1);
        if (lane == 0) Jp = Jprev;
        const bool start = valid && J != Jp;
        const unsigned long long sm = __ballot(start);
        if (start) {
            const unsigned long long nx = sm & above;
            int64_t len;
            if (nx)
                len = __ffsll((long long)nx) - 1 - lane;
            else   // the chunk's last segment: to the chunk's end, then on
                len = min<int64_t>(e, c0 + kWave) - p + __popcll(cont);
            const int64_t tt = tbI + w.y + __popc(w.x & ((1u << (d & 31)) - 1u));
            seg[tt * kTile + r] = (p << 5) | len;
        }
        Jprev = Jlast;
        J = Jn;
    }
}

// One wave per tile: the tile is assembled in LDS in both operand layouts
// (the B layout only when tA is NULL) from its row segments (16 lanes per
// row, consecutive entries) and written out whole, 32 contiguous bytes per
// lane.
__global__ __launch_bounds__(256) void k_bsr_assemble(CsrView T, int64_t ntiles,
                                                      const int32_t *tcols, const int32_t *trows,
                                                      const int64_t *seg, double *tA,
                                                      double *tB) {
    __shared__ double buf[4][2][kTileElems];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t tt = (int64_t)blockIdx.x * 4 + wv;
    if (tt >= ntiles) return;
    double *bA = buf[wv][0], *bB = buf[wv][1];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        bA[4 * lane + q] = 0.0;
        bB[4 * lane + q] = 0.0;
    }
    wfence();
    // rows past the matrix have no segment (the table starts zeroed), so the
    // segment loads need nothing else first
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int r = 4 * rr + (lane >> 4);
        const int64_t s = seg[tt * kTile + r];
        const int j = lane & 15;
        if (j < (int)(s & 31)) {
            const int64_t p = (s >> 5) + j;
            const int c = T.ci[p] & 15;
            const double v = T.v[p];
            if (tA) bA[offA(r, c)] = v;
            bB[offB(r, c)] = v;
        }
    }
    wfence();
    if (tA) *(d4 *)(tA + tt * kTileElems + 4 * lane) = *(const d4 *)(bA + 4 * lane);
    *(d4 *)(tB + tt * kTileElems + 4 * lane) = *(const d4 *)(bB + 4 * lane);
    (void)tcols;
    (void)trows;
}

// For a symmetric tile pattern: mir[t] = the index of tile t's transpose
// (block row and column exchanged).  A missing transpose sets *bad and
// leaves 0, a valid index.
__global__ void k_bsr_tile_mirrors(int64_t ntiles, const int32_t *lo, const int64_t *woff,
                                   const uint2 *rt, const int64_t *tb, const int32_t *tcols,
                                   const int32_t *trows, int64_t *mir, int *bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t m = tile_of(lo, woff, rt, tb, tcols[t], trows[t]);
    if (m < 0) atomicOr(bad, 1);
    mir[t] = m < 0 ? 0 : m;
}

hipError_t bsr_tile_mirrors(int64_t ntiles, const int32_t *lo, const int64_t *woff,
                            const uint2 *rt, const int64_t *tb, const int32_t *tcols,
                            const int32_t *trows, int64_t *mir, int *bad, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_tile_mirrors, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0,
                       st, ntiles, lo, woff, rt, tb, tcols, trows, mir, bad);
    return hipGetLastError();
}

// ----------------------------------------------------------------- C pattern

// Block-column range of C's block row I: the union of T's block rows K for
// the block columns K of block row I (and block row I itself, the 2T term).
__global__ void k_bsr_cbounds(int64_t nb, const int32_t *lo, const int64_t *woff,
                              const uint2 *rt, const int64_t *tb, int32_t *clo,
                              int64_t *cwords) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= nb) return;
    const int lane = lane_id();
    const int64_t W = woff[I + 1] - woff[I];
    int mn = INT32_MAX, mx = -1;
    if (W > 0) {
        mn = lo[I];
        mx = lo[I] + 32 * (int)W - 1;
    }
    // every set bit of block row I names a block row K
    for (int64_t w = lane; w < W; w += kWave) {
        uint32_t x = rt[woff[I] + w].x;
        while (x) {
            const int K = lo[I] + 32 * (int)w + __ffs(x) - 1;
            x &= x - 1;
            const int64_t WK = woff[K + 1] - woff[K];
            if (WK > 0) {
                mn = min(mn, lo[K]);
                mx = max(mx, lo[K] + 32 * (int)WK - 1);
            }
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0) {
        if (mx < 0) {
            clo[I] = 0;
            cwords[I] = 0;
        } else {
            clo[I] = mn;
            cwords[I] = ((mx - mn) >> 5) + 1;
        }
    }
}

// C's block-row bit maps (word-aligned ORs of T's bit maps) and tile counts;
// with ccols != NULL also the sorted block-column list of every C block row
// and C's rank table crt (word, prefix count), as T's rt.
__global__ __launch_bounds__(64) void k_bsr_cpattern(int64_t nb, const int32_t *lo,
                                                     const int64_t *woff, const uint2 *rt,
                                                     const int32_t *clo, const int64_t *cwoff,
                                                     int64_t *ccnt, const int64_t *ctb,
                                                     int32_t *ccols, uint2 *crt) {
    extern __shared__ uint32_t bm[];
    const int64_t I = blockIdx.x;
    if (I >= nb) return;
    const int lane = lane_id();
    const int64_t CW = cwoff[I + 1] - cwoff[I];
    if (CW == 0) {
        if (lane == 0 && !ccols) ccnt[I] = 0;
        return;
    }
    for (int64_t w = lane; w < CW; w += kWave) bm[w] = 0;
    wfence();
    const int cbase = clo[I];
    auto or_row = [&](int64_t K) {
        const int64_t WK = woff[K + 1] - woff[K];
        const int sh = (lo[K] - cbase) >> 5;   // both origins are multiples of 32
        for (int64_t w = lane; w < WK; w += kWave) {
            const uint32_t x = rt[woff[K] + w].x;
            if (x) atomicOr(&bm[sh + w], x);
        }
    };
    or_row(I);
    const int64_t W = woff[I + 1] - woff[I];
    for (int64_t w = 0; w < W; ++w) {
        uint32_t x = rt[woff[I] + w].x;
        while (x) {
            const int K = lo[I] + 32 * (int)w + __ffs(x) - 1;
            x &= x - 1;
            or_row(K);
        }
    }
    wfence();
    unsigned carry = 0;
    for (int64_t b0 = 0; b0 < CW; b0 += kWave) {
        const int64_t w = b0 + lane;
        uint32_t x = w < CW ? bm[w] : 0u;
        const unsigned pc = __popc(x);
        const unsigned inc = wave_incl_scan(pc);
        if (ccols && w < CW) {
            unsigned r = carry + inc - pc;
            crt[cwoff[I] + w] = make_uint2(x, r);
            while (x) {
                ccols[ctb[I] + r] = cbase + 32 * (int)w + __ffs(x) - 1;
                x &= x - 1;
                ++r;
            }
        }
        carry += __shfl(inc, kWave - 1);
    }
    if (lane == 0 && !ccols) ccnt[I] = carry;
}

__global__ void k_bsr_groups(const int64_t *ccnt, int64_t nb, int64_t *gcnt, int group) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nb) gcnt[I] = (ccnt[I] + group - 1) / group;
}

// owner[w] = i for every work item w in [ofs[i], ofs[i + 1]) (ofs: the
// exclusive scan of the work-item counts, ofs[m] the total), so that a work
// item finds its panel or block row with one load instead of a binary
// search of dependent loads.
__global__ void k_work_owner(const int64_t *ofs, int64_t m, int32_t *owner) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t w = ofs[i]; w < ofs[i + 1]; ++w) owner[w] = (int32_t)i;
}

// ----------------------------------------------------------------- product

// ----------------------------------------------------------------- panels
//
// A panel is kPanel consecutive block rows of C.  Its four waves (one block
// row each) take the same kPanelGroup block columns from the union of the
// panel's C patterns, so for every K they read the same B tiles T_KJ close
// together in time and share them through the CU's caches; each wave reads
// its own A tiles.  Output tiles absent from a row's C pattern receive no
// product and are not written.

// Panel origin (block column, multiple of 32) and bit-map words.
__global__ void k_panel_bounds(int64_t nb, const int32_t *clo, const int64_t *cwoff,
                               int32_t *plo, int64_t *pwords) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (nb + kPanel - 1) / kPanel;
    if (p >= np) return;
    int mn = INT32_MAX, mx = -1;
    for (int64_t I = p * kPanel; I < min<int64_t>(p * kPanel + kPanel, nb); ++I) {
        const int64_t CW = cwoff[I + 1] - cwoff[I];
        if (CW > 0) {
            mn = min(mn, clo[I]);
            mx = max(mx, clo[I] + 32 * (int)CW - 1);
        }
    }
    if (mx < 0) {
        plo[p] = 0;
        pwords[p] = 0;
    } else {
        plo[p] = mn;
        pwords[p] = ((mx - mn) >> 5) + 1;
    }
}

// Union of the C block-column lists of a panel: counts (pcols == NULL) or
// the sorted list at pofs[p].  With upper, only the block columns at or
// right of the panel's first block row (a symmetric C is formed from its
// upper triangle).
__global__ __launch_bounds__(64) void k_panel_cols(int64_t nb, const int32_t *clo,
                                                   const int64_t *cwoff, const uint2 *crt,
                                                   const int32_t *plo, const int64_t *pwoff,
                                                   int64_t *pcnt, const int64_t *pofs,
                                                   int32_t *pcols, int upper) {
    extern __shared__ uint32_t bm[];
    const int64_t p = blockIdx.x;
    const int lane = lane_id();
    const int64_t PW = pwoff[p + 1] - pwoff[p];
    if (PW == 0) {
        if (lane == 0 && !pcols) pcnt[p] = 0;
        return;
    }
    for (int64_t w = lane; w < PW; w += kWave) bm[w] = 0;
    wfence();
    for (int64_t I = p * kPanel; I < min<int64_t>(p * kPanel + kPanel, nb); ++I) {
        const int64_t CW = cwoff[I + 1] - cwoff[I];
        const int sh = (clo[I] - plo[p]) >> 5;
        for (int64_t w = lane; w < CW; w += kWave) {
            const uint32_t x = crt[cwoff[I] + w].x;
            if (x) atomicOr(&bm[sh + w], x);
        }
    }
    wfence();
    const int base = plo[p];
    const int64_t first = upper ? p * kPanel : INT32_MIN;   // smallest block column kept
    unsigned carry = 0;
    for (int64_t b0 = 0; b0 < PW; b0 += kWave) {
        const int64_t w = b0 + lane;
        uint32_t x = w < PW ? bm[w] : 0u;
        const int64_t c0 = base + 32 * w;   // block column of bit 0
        if (c0 + 32 <= first)
            x = 0u;
        else if (c0 < first)
            x &= ~((1u << (unsigned)(first - c0)) - 1u);
        const unsigned pc = __popc(x);
        const unsigned inc = wave_incl_scan(pc);
        if (pcols && w < PW) {
            unsigned r = carry + inc - pc;
            while (x) {
                pcols[pofs[p] + r] = base + 32 * (int)w + __ffs(x) - 1;
                x &= x - 1;
                ++r;
            }
        }
        carry += __shfl(inc, kWave - 1);
    }
    if (lane == 0 && !pcols) pcnt[p] = carry;
}

// The end of a panel work item: each output tile t < ng with act[t] that is
// in C's pattern is written (streaming stores) with its summaries; with
// upper its transpose too, passed through the wave's LDS tile M.
template <int kGroup>
__device__ __forceinline__ void panel_epilogue(
    int64_t I, int ng, const int (&J)[kGroup], const bool (&act)[kGroup], const d4 (&acc)[kGroup],
    const int32_t *__restrict__ clo, const int64_t *__restrict__ cwoff,
    const uint2 *__restrict__ crt, const int64_t *__restrict__ ctb, double *__restrict__ ctiles,
    int64_t n, double *__restrict__ tsq, int32_t *__restrict__ tnz, double *__restrict__ tmn,
    double *__restrict__ tmx, uint4 *__restrict__ trc, double *__restrict__ bdg, int upper,
    int *__restrict__ bad, int64_t *__restrict__ tmir, double *M) {
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        if (t >= ng) break;
        if (!act[t]) continue;
        const int64_t ct = tile_of(clo, cwoff, crt, ctb, I, J[t]);
        if (ct < 0) continue;
        // candidate tiles are written once and read back by later kernels,
        // after far more data than the caches hold has passed: streaming
        // stores keep them from displacing the operand tiles still in use
        __builtin_nontemporal_store(acc[t], (d4 *)(ctiles + ct * kTileElems + 4 * lane));
        // with upper, tile (J, I) left of the diagonal is this one's
        // transpose: lane holds (4 k + lane / 16, lane % 16) of it, i.e.
        // (lane % 16, 4 k + lane / 16) of acc
        int64_t ctT = -1;
        uint32_t rcT[4] = {0u, 0u, 0u, 0u};
        if (upper && J[t] != (int)I) {
            ctT = tile_of(clo, cwoff, crt, ctb, J[t], (int)I);
            if (ctT < 0) {
                if (lane == 0) atomicOr(bad, 1);
            } else {
                const int g = lane >> 4, c = lane & 15;
#pragma unroll
                for (int k = 0; k < 4; ++k) M[(4 * k + g) * (kTile + 1) + c] = acc[t][k];
                wfence();
                d4 u;
#pragma unroll
                for (int k = 0; k < 4; ++k) u[k] = M[c * (kTile + 1) + 4 * k + g];
                wfence();
                __builtin_nontemporal_store(u, (d4 *)(ctiles + ctT * kTileElems + 4 * lane));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned long long m = __ballot(u[r] != 0.0);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rcT[r] |= (uint32_t)__popcll((m >> (16 * q)) & 0xffffull) << (8 * q);
                }
            }
        }
        if (!tsq) continue;
        // the tile's sum of squares, its nonzero slots, their smallest and
        // largest magnitudes and the nonzeros of each of its 16 rows, all
        // over the rows below n (slots outside the matrix hold zeros); for
        // the diagonal tile also sum (2 c_ii + 1), which turns its share of
        // ||C||_F^2 into its share of ||I + C||_F^2.  Lane holds
        // (i, j) = (4 r + lane / 16, lane % 16).
        const int rows = (int)min<int64_t>(kTile, n - I * kTile);
        const bool dtile = J[t] == (int)I;
        double s = 0.0, mn = INFINITY, mx = 0.0, dg = 0.0;
        long long nz = 0;
        uint32_t rc[4] = {0u, 0u, 0u, 0u};   // byte i % 4 of word i / 4: row i
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * r + (lane >> 4);
            const bool in = i < rows;
            const double v = in ? acc[t][r] : 0.0;
            s = fma(v, v, s);
            if (in && i == (lane & 15)) dg += fma(2.0, v, 1.0);
            nz += v != 0.0;
            if (v != 0.0) mn = fmin(mn, fabs(v));
            mx = fmax(mx, fabs(v));
            // rows 4 r .. 4 r + 3 are the four 16-lane groups of register r
            const unsigned long long m = __ballot(v != 0.0);
#pragma unroll
            for (int g = 0; g < 4; ++g)
                rc[r] |= (uint32_t)__popcll((m >> (16 * g)) & 0xffffull) << (8 * g);
        }
        s = wave_sum(s);
        nz = wave_sum_ll(nz);
        mn = wave_min_f64(mn);
        mx = wave_max_f64(mx);
        if (dtile) {
            dg = wave_sum(dg);
            if (lane == 0) bdg[I] = dg;
        }
        if (lane == 0) {
            tsq[ct] = s;
            tnz[ct] = (int32_t)nz;
            tmn[ct] = mn;
            tmx[ct] = mx;
            trc[ct] = make_uint4(rc[0], rc[1], rc[2], rc[3]);
            if (ctT >= 0) {   // the transpose: same values, its own row counts
                tsq[ctT] = s;
                tnz[ctT] = (int32_t)nz;
                tmn[ctT] = mn;
                tmx[ctT] = mx;
                trc[ctT] = make_uint4(rcT[0], rcT[1], rcT[2], rcT[3]);
            }
            if (tmir) {   // the pairing the filter passes use
                tmir[ct] = ctT >= 0 ? ctT : -1;
                if (ctT >= 0) tmir[ctT] = -2;
            }
        }
    }
}

// One workgroup per work item (panel, group of kGroup panel columns); wave
// w computes block row kPanel p + w.  C_IJ = (2 I) T_IJ + sum_K T_IK T_KJ
// with K ascending over the tiles of T's block row I.  The lanes first find,
// 64 values of K at a time, the tiles T_KJ of the group (one K per lane, all
// lookups in flight together); the product loop then walks the K that have
// at least one, reading their indices with readlane, and loads the operands
// of the next K before issuing the matrix instructions of the current one.
// The kernel waits on the latency of its operand loads far more than on the
// matrix cores, so it takes two output tiles per wave and is held to 80
// registers: six waves per SIMD keep more loads in flight than four waves
// of four tiles (128 registers) or eight of one.
// With upper (a symmetric T, hence a symmetric C) the panels' column lists
// start at the panel's first block row, each wave skips the tiles left of
// its diagonal, and every off-diagonal tile it forms is also written,
// transposed through LDS, to the mirror tile left of the diagonal (with
// the same sum of squares, nonzero count and magnitudes, and that tile's
// own per-row counts).
template <int kGroup>
__global__ __launch_bounds__(kWave * kPanel)
__attribute__((amdgpu_waves_per_eu(6))) void k_bsr_numeric_panel(
    int64_t nb, const int32_t *__restrict__ lo, const int64_t *__restrict__ woff,
    const uint2 *__restrict__ rt, const int64_t *__restrict__ tb,
    const int32_t *__restrict__ tcols, const double *__restrict__ tA,
    const double *__restrict__ tB, const int64_t *__restrict__ pgofs,
    const int64_t *__restrict__ nwork_dev, const int32_t *__restrict__ owner,
    const int64_t *__restrict__ pofs, const int32_t *__restrict__ pcols,
    const int32_t *__restrict__ clo, const int64_t *__restrict__ cwoff,
    const uint2 *__restrict__ crt, const int64_t *__restrict__ ctb, double *__restrict__ ctiles,
    int64_t n, double *__restrict__ tsq, int32_t *__restrict__ tnz, double *__restrict__ tmn,
    double *__restrict__ tmx, uint4 *__restrict__ trc, double *__restrict__ bdg, int upper,
    int *__restrict__ bad, int64_t *__restrict__ tmir, const int64_t *__restrict__ amir,
    int xcd) {
    // with upper: one transposed tile per wave passes through LDS (rows
    // padded to 17 doubles)
    __shared__ double tsm[kPanel][kTile * (kTile + 1)];
    const int lane = lane_id();
    const int64_t nw = *nwork_dev;
    const int64_t w = xcd ? xcd_item(blockIdx.x, nw) : (int64_t)blockIdx.x;
    if (w < 0 || w >= nw) return;
    const int64_t p = owner[w];   // the panel: pgofs[p] <= w < pgofs[p + 1]
    const int64_t I = p * kPanel + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (I >= nb) return;
    const int64_t g0 = (w - pgofs[p]) * kGroup;
    const int ng = (int)min<int64_t>(kGroup, pofs[p + 1] - pofs[p] - g0);
    int J[kGroup];
    // with upper, the tiles left of the diagonal are not formed here (they
    // are the transposes of tiles right of it)
    bool act[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        J[t] = t < ng ? pcols[pofs[p] + g0 + t] : -1;
        act[t] = t < ng && (!upper || J[t] >= (int)I);
    }
    d4 acc[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    {
        const d4 two = two_identity_a(lane);
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
            if (t >= ng) break;
            if (!act[t]) continue;
            const int64_t tt = tile_of(lo, woff, rt, tb, I, J[t]);
            if (tt < 0) continue;
            const d4 b = *(const d4 *)(tB + tt * kTileElems + 4 * lane);
            acc[t] = mfma16(two, b, acc[t]);
        }
    }
    const int64_t t0 = tb[I], nk = tb[I + 1] - t0;
    const int jlo = J[0], jhi = last_of(J, ng);
    // A operand T_IK: tile t0 + r in the A layout, or, for a symmetric T
    // assembled in the B layout only (amir), the B layout of its transpose
    auto item = [&](int64_t r, int &K, int &a) {
        K = tcols[t0 + r];
        a = amir ? (int)amir[t0 + r] : (int)(t0 + r);
    };
    auto look = [&](int K, int (&ti)[kGroup]) {
        const int loK = lo[K];
        const int64_t w0 = woff[K], WK = woff[K + 1] - w0;
        if (WK == 0 || jhi < loK || jlo >= loK + 32 * (int)WK) return;
        const int64_t tbK = tb[K];
#pragma unroll
        for (int t = 0; t < kGroup; ++t)
            if (act[t]) ti[t] = tile_in_row(loK, w0, WK, tbK, rt, J[t]);
    };
    pipe_products<kGroup>(nk, item, look, tA, tB, acc);
    panel_epilogue<kGroup>(I, ng, J, act, acc, clo, cwoff, crt, ctb, ctiles, n, tsq, tnz, tmn, tmx,
                           trc, bdg, upper, bad, tmir, tsm[threadIdx.x / kWave]);
}

// ----------------------------------------------------------------- norm, compaction

// Per block row, from the per-tile partials the product wrote: the sum over
// its candidate slots of (c_ij + delta_ij)^2 for the rows below n (the
// tiles' sums of squares, plus the diagonal tile's sum of (2 c_ii + 1), or
// plus 1 for each row when that tile is absent); and the count of nonzero
// slots.  Tiles are taken lane-strided in index order, then a fixed
// butterfly, so the result is reproducible.
__global__ void k_bsr_norm_tiles(int64_t n, int64_t nb, const int64_t *ctb, const int64_t *ccnt,
                                 const int32_t *ccols, const double *tsq, const int32_t *tnz,
                                 const double *bdg, double *bsq, int64_t *bnz) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= nb) return;
    const int lane = lane_id();
    const int rows = (int)min<int64_t>(kTile, n - I * kTile);
    const int64_t b = ctb[I], e = b + ccnt[I];
    double s = 0.0;
    long long nz = 0;
    bool diag = false;
    for (int64_t t = b + lane; t < e; t += kWave) {
        s += tsq[t];
        nz += tnz[t];
        diag |= ccols[t] == (int)I;
    }
    s = wave_sum(s);
    nz = wave_sum_ll(nz);
    diag = __ballot(diag) != 0ull;
    if (lane == 0) {
        bsq[I] = diag ? s + bdg[I] : s + rows;
        bnz[I] = nz;
    }
}

// Compaction of the candidate tiles.  One wave per block row I reads each
// tile of the block row once (32 contiguous bytes per lane): lane l holds
// column l % 16 of rows r = l / 16 + 4 k, k = 0..3 (the accumulator layout),
// so the 16 lanes of group g = l / 16 see the full 16 columns of rows g,
// g + 4, g + 8, g + 12.  An entry is kept when its row and column are below
// n and |v| > theta; tiles run in ascending block column, so each row's kept
// entries come out in column order.
__device__ __forceinline__ bool bsr_keep(int64_t i, int col, int64_t n, double v, double theta) {
    return i < n && col < n && fabs(v) > theta;
}

// With the per-tile summaries of the product (tmn, tmx: smallest nonzero and
// largest magnitude, trc: nonzeros per row), a tile whose slots are all at
// most theta is skipped, and one whose nonzeros all exceed theta is counted
// from trc without reading it; with krc, the tiles in between are counted
// from the last filter pass's counts, so no tile is read.  With rcnt, the
// kept entries of each of the 16 rows in each round of 64 tiles too, at
// rcnt[(rofs[I] + round) * 16 + row] (for k_bsr_write_rounds).
__global__ void k_bsr_count(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                            const int32_t *ccols, const double *ctiles, const double *tmn,
                            const double *tmx, const uint4 *trc, const uint4 *krc,
                            const FilterCtl *c, int64_t *cnt, int32_t *rcnt,
                            const int64_t *rofs) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= (n + kTile - 1) / kTile) return;
    const int lane = lane_id();
    const int g = lane >> 4;
    const double theta = c->theta;
    int k4[4] = {0, 0, 0, 0};   // kept per row, reduced over the 16 lanes of each group
    const int64_t base = ctb[I], cntI = ccnt[I];
    for (int64_t c0 = 0; c0 < cntI; c0 += kWave) {
        int r4[4] = {0, 0, 0, 0};   // this round's, per lane
        // one lane per tile: the summaries of 64 tiles are read together;
        // h holds the row counts in 16-bit fields, row r in half r & 1 of
        // word r >> 1 (at most 16 per tile, 1024 per round)
        const int64_t t = c0 + lane, tt = base + t;
        uint32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        bool rd = false;
        if (t < cntI) {
            if (!tmx) {
                rd = true;
            } else if (tmx[tt] > theta) {
                const bool whole = tmn[tt] > theta;
                if (whole || krc) {
                    // wholly kept: the product's row counts; in between:
                    // the counts the last filter pass took at this threshold
                    const uint4 q = whole ? trc[tt] : krc[tt];
                    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k)
#pragma unroll
                        for (int gg = 0; gg < 4; ++gg) {
                            const int row = gg + 4 * k;
                            h[row >> 1] += ((w[k] >> (8 * gg)) & 0xffu) << (16 * (row & 1));
                        }
                } else {
                    rd = true;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) h[j] += __shfl_xor(h[j], o);
        if ((lane & 15) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int row = g + 4 * k;
                r4[k] += (int)((h[row >> 1] >> (16 * (row & 1))) & 0xffffu);
            }
        }
        // tiles without usable counts are read, one at a time by all lanes
        unsigned long long m = __ballot(rd);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int64_t tr = base + c0 + l;
            const int col = 16 * ccols[tr] + (lane & 15);
            const d4 v = *(const d4 *)(ctiles + tr * kTileElems + 4 * lane);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                r4[k] += bsr_keep(I * kTile + g + 4 * k, col, n, v[k], theta);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) r4[k] += __shfl_xor(r4[k], o);
            k4[k] += r4[k];
        }
        if (rcnt && (lane & 15) == 0) {
            const int64_t q = rofs[I] + c0 / kWave;
#pragma unroll
            for (int k = 0; k < 4; ++k) rcnt[q * kTile + g + 4 * k] = r4[k];
        }
    }
    if ((lane & 15) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = I * kTile + g + 4 * k;
            if (i < n) cnt[i] = k4[k];
        }
    }
}

__global__ void k_bsr_write(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                            const int32_t *ccols, const double *ctiles, const double *tmx,
                            const FilterCtl *c, const int64_t *orp, int32_t *oci, double *ov) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= (n + kTile - 1) / kTile) return;
    const int lane = lane_id();
    const int g = lane >> 4, cl = lane & 15;
    const double theta = c->theta;
    int64_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = I * kTile + g + 4 * k;
        out[k] = i < n ? orp[i] : 0;
    }
    const int64_t base = ctb[I], cntI = ccnt[I];
    const uint32_t below = (1u << cl) - 1u;
    auto emit = [&](int col, const d4 &v) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool keep = bsr_keep(I * kTile + g + 4 * k, col, n, v[k], theta);
            const uint32_t gm = (uint32_t)(__ballot(keep) >> (16 * g)) & 0xffffu;
            if (keep) {
                const int64_t q = out[k] + __popc(gm & below);
                oci[q] = col;
                ov[q] = v[k];
            }
            out[k] += __popc(gm);
        }
    };
    for (int64_t c0 = 0; c0 < cntI; c0 += kWave) {
        // one lane per tile: which of 64 tiles keep anything, and their block
        // columns, in one round trip; then the tiles that do, in order, with
        // the loads of the next two in flight while the current one is written
        const int64_t t = c0 + lane;
        const bool some = t < cntI && (!tmx || tmx[base + t] > theta);
        const int bc = some ? ccols[base + t] : 0;
        unsigned long long m = __ballot(some);
        auto pop = [&](int &col, d4 &v) {
            if (!m) return false;
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            col = 16 * __builtin_amdgcn_readlane(bc, l) + cl;
            v = *(const d4 *)(ctiles + (base + c0 + l) * kTileElems + 4 * lane);
            return true;
        };
        int col0 = 0, col1 = 0;
        d4 v0 = d4{0.0, 0.0, 0.0, 0.0}, v1 = v0;
        bool h0 = pop(col0, v0);
        bool h1 = pop(col1, v1);
        while (h0) {
            int col2 = 0;
            d4 v2 = d4{0.0, 0.0, 0.0, 0.0};
            const bool h2 = pop(col2, v2);
            emit(col0, v0);
            col0 = col1;
            v0 = v1;
            h0 = h1;
            col1 = col2;
            v1 = v2;
            h1 = h2;
        }
    }
}

// k_bsr_write with one wave per round of 64 tiles of a block row (work item
// w: block row owner[w], round w - rofs[I]) instead of one per block row, so
// that a long block row is written by several waves at once: each round's
// rows start after the kept entries that k_bsr_count found in the row's
// earlier rounds (rcnt).
__global__ void k_bsr_write_rounds(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                                   const int32_t *ccols, const double *ctiles, const double *tmx,
                                   const FilterCtl *c, const int64_t *orp, const int32_t *rcnt,
                                   const int64_t *rofs, const int32_t *owner,
                                   const int64_t *nwork_dev, int32_t *oci, double *ov) {
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (w >= *nwork_dev) return;
    const int64_t I = owner[w];
    const int64_t q = w - rofs[I];
    const int lane = lane_id();
    const int g = lane >> 4, cl = lane & 15;
    const double theta = c->theta;
    int64_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = I * kTile + g + 4 * k;
        int64_t o = i < n ? orp[i] : 0;
        for (int64_t qq = 0; qq < q; ++qq) o += rcnt[(rofs[I] + qq) * kTile + g + 4 * k];
        out[k] = o;
    }
    const int64_t base = ctb[I], cntI = ccnt[I];
    const uint32_t below = (1u << cl) - 1u;
    auto emit = [&](int col, const d4 &v) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool keep = bsr_keep(I * kTile + g + 4 * k, col, n, v[k], theta);
            const uint32_t gm = (uint32_t)(__ballot(keep) >> (16 * g)) & 0xffffu;
            if (keep) {
                const int64_t p = out[k] + __popc(gm & below);
                oci[p] = col;
                ov[p] = v[k];
            }
            out[k] += __popc(gm);
        }
    };
    // the round's tiles: which of them keep anything, and their block
    // columns, in one round trip; then those that do, in order, with the
    // loads of the next two in flight while the current one is written
    const int64_t c0 = q * kWave, t = c0 + lane;
    const bool some = t < cntI && (!tmx || tmx[base + t] > theta);
    const int bc = some ? ccols[base + t] : 0;
    unsigned long long m = __ballot(some);
    auto pop = [&](int &col, d4 &v) {
        if (!m) return false;
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        col = 16 * __builtin_amdgcn_readlane(bc, l) + cl;
        v = *(const d4 *)(ctiles + (base + c0 + l) * kTileElems + 4 * lane);
        return true;
    };
    int col0 = 0, col1 = 0;
    d4 v0 = d4{0.0, 0.0, 0.0, 0.0}, v1 = v0;
    bool h0 = pop(col0, v0);
    bool h1 = pop(col1, v1);
    while (h0) {
        int col2 = 0;
        d4 v2 = d4{0.0, 0.0, 0.0, 0.0};
        const bool h2 = pop(col2, v2);
        emit(col0, v0);
        col0 = col1;
        v0 = v1;
        h0 = h1;
        col1 = col2;
        v1 = v2;
        h1 = h2;
    }
}

// Per row i < n of the candidate: sum over the row's tile slots of
// (c_ij + delta_ij)^2, plus 1 when the row's diagonal tile is absent (its
// row's contribution to ||I + C||_F^2; padding slots hold zeros).
__global__ void k_bsr_rowsq(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                            const int32_t *ccols, const double *ctiles, double *rowsq) {
    const int64_t I = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (I >= (n + kTile - 1) / kTile) return;
    const int lane = lane_id();
    const int g = lane >> 4, cl = lane & 15;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    bool diag = false;
    const int64_t base = ctb[I], cntI = ccnt[I];
    for (int64_t t = 0; t < cntI; ++t) {
        const int64_t tt = base + t;
        const bool dtile = ccols[tt] == (int)I;
        diag |= dtile;
        const d4 v = *(const d4 *)(ctiles + tt * kTileElems + 4 * lane);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double f = dtile && g + 4 * k == cl ? v[k] + 1.0 : v[k];
            s4[k] = fma(f, f, s4[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) s4[k] += __shfl_xor(s4[k], o);
    if (cl == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = I * kTile + g + 4 * k;
            if (i < n) rowsq[i] = diag ? s4[k] : s4[k] + 1.0;
        }
    }
}

// ----------------------------------------------------------------- host wrappers

size_t bsr_lds_words(int64_t n) { return (size_t)((n + 15) / 16 + 31) / 32 + 2; }

hipError_t bsr_bounds(CsrView T, int64_t nb, int32_t *lo, int64_t *words, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_bounds, dim3((nb + 3) / 4), dim3(256), 0, st, T, nb, lo, words);
    return hipGetLastError();
}

hipError_t bsr_bitmap(CsrView T, int64_t nb, const int32_t *lo, const int64_t *woff, uint2 *rt,
                      int64_t *cnt, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_bitmap, dim3(nb), dim3(64), bsr_lds_words(T.n) * 4, st, T, nb, lo,
                       woff, rt, cnt);
    return hipGetLastError();
}

hipError_t bsr_cbounds(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                       const int64_t *tb, int32_t *clo, int64_t *cwords, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_cbounds, dim3((nb + 3) / 4), dim3(256), 0, st, nb, lo, woff, rt, tb,
                       clo, cwords);
    return hipGetLastError();
}

hipError_t bsr_cpattern(int64_t n, int64_t nb, const int32_t *lo, const int64_t *woff,
                        const uint2 *rt, const int32_t *clo, const int64_t *cwoff, int64_t *ccnt,
                        const int64_t *ctb, int32_t *ccols, uint2 *crt, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_cpattern, dim3(nb), dim3(64), bsr_lds_words(n) * 4, st, nb, lo,
                       woff, rt, clo, cwoff, ccnt, ctb, ccols, crt);
    return hipGetLastError();
}

hipError_t bsr_panel_bounds(int64_t nb, const int32_t *clo, const int64_t *cwoff, int32_t *plo,
                            int64_t *pwords, hipStream_t st) {
    const int64_t np = (nb + kPanel - 1) / kPanel;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_panel_bounds, dim3((np + 255) / 256), dim3(256), 0, st, nb, clo, cwoff,
                       plo, pwords);
    return hipGetLastError();
}

hipError_t bsr_panel_cols(int64_t n, int64_t nb, const int32_t *clo, const int64_t *cwoff,
                          const uint2 *crt, const int32_t *plo, const int64_t *pwoff,
                          int64_t *pcnt, const int64_t *pofs, int32_t *pcols, hipStream_t st,
                          bool upper) {
    const int64_t np = (nb + kPanel - 1) / kPanel;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_panel_cols, dim3((unsigned)np), dim3(64), bsr_lds_words(n) * 4, st, nb,
                       clo, cwoff, crt, plo, pwoff, pcnt, pofs, pcols, upper ? 1 : 0);
    return hipGetLastError();
}

int64_t bsr_panel_work_bound(int64_t ctiles, int64_t nb) {
    // a panel's union holds at most the sum of its rows' tiles, and each
    // panel rounds up once
    return ctiles / kPanelGroup + (nb + kPanel - 1) / kPanel + 1;
}

hipError_t bsr_panel_groups(const int64_t *pcnt, int64_t nb, int64_t *gcnt, hipStream_t st) {
    const int64_t np = (nb + kPanel - 1) / kPanel;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_groups, dim3((np + 255) / 256), dim3(256), 0, st, pcnt, np, gcnt,
                       kPanelGroup);
    return hipGetLastError();
}

hipError_t work_owner(const int64_t *ofs, int64_t m, int32_t *owner, hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_work_owner, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, ofs, m,
                       owner);
    return hipGetLastError();
}

hipError_t bsr_tcols(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                     const int64_t *tb, int32_t *tcols, int32_t *trows, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_tcols, dim3((nb + 3) / 4), dim3(256), 0, st, nb, lo, woff, rt, tb,
                       tcols, trows);
    return hipGetLastError();
}

hipError_t bsr_seg(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                   const int64_t *tb, int64_t *seg, hipStream_t st) {
    if (T.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_seg, dim3((T.n + 3) / 4), dim3(256), 0, st, T, lo, woff, rt, tb, seg);
    return hipGetLastError();
}

hipError_t bsr_assemble(CsrView T, int64_t ntiles, const int32_t *tcols, const int32_t *trows,
                        const int64_t *seg, double *tA, double *tB, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_assemble, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, T,
                       ntiles, tcols, trows, seg, tA, tB);
    return hipGetLastError();
}

hipError_t bsr_numeric_panel(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                             const int64_t *tb, const int32_t *tcols, const double *tA,
                             const double *tB, const int64_t *pgofs, const int64_t *nwork_dev,
                             const int32_t *owner, const int64_t *pofs, const int32_t *pcols,
                             const int32_t *clo, const int64_t *cwoff, const uint2 *crt,
                             const int64_t *ctb, double *ctiles, int64_t n, double *tsq,
                             int32_t *tnz, double *tmn, double *tmx, uint4 *trc, double *bdg,
                             int64_t nwork, hipStream_t st, bool upper, int *bad,
                             int64_t *tmir, const int64_t *amir) {
    if (nwork == 0) return hipSuccess;
    // work items spread over the XCDs in contiguous ranges (EXPM_TILE_XCD=0:
    // round robin, the hardware's order)
    static const int xcd = [] {
        const char *e = getenv("EXPM_TILE_XCD");
        return e && e[0] == '0' ? 0 : 1;
    }();
    hipLaunchKernelGGL(k_bsr_numeric_panel<kPanelGroup>, dim3((unsigned)(nwork + 8)),
                       dim3(kWave * kPanel), 0, st, nb, lo, woff, rt, tb, tcols,
                       amir ? tB : tA, tB, pgofs, nwork_dev, owner, pofs, pcols, clo, cwoff, crt,
                       ctb, ctiles, n, tsq, tnz, tmn, tmx, trc, bdg, upper ? 1 : 0, bad, tmir,
                       amir, xcd);
    return hipGetLastError();
}

hipError_t bsr_norm_tiles(int64_t n, int64_t nb, const int64_t *ctb, const int64_t *ccnt,
                          const int32_t *ccols, const double *tsq, const int32_t *tnz,
                          const double *bdg, double *bsq, int64_t *bnz, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_norm_tiles, dim3((nb + 3) / 4), dim3(256), 0, st, n, nb, ctb, ccnt,
                       ccols, tsq, tnz, bdg, bsq, bnz);
    return hipGetLastError();
}

hipError_t bsr_rowsq(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, double *rowsq, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_bsr_rowsq, dim3((nb + 3) / 4), dim3(256), 0, st, n, ctb, ccnt, ccols,
                       ctiles, rowsq);
    return hipGetLastError();
}

hipError_t bsr_count(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, const double *tmn, const double *tmx,
                     const uint4 *trc, const uint4 *krc, const FilterCtl *c, int64_t *cnt,
                     hipStream_t st, int32_t *rcnt, const int64_t *rofs) {
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_bsr_count, dim3((nb + 3) / 4), dim3(256), 0, st, n, ctb, ccnt, ccols,
                       ctiles, tmn, tmx, trc, krc, c, cnt, rcnt, rofs);
    return hipGetLastError();
}

hipError_t bsr_write_rounds(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                            const int32_t *ccols, const double *ctiles, const double *tmx,
                            const FilterCtl *c, const int64_t *orp, const int32_t *rcnt,
                            const int64_t *rofs, const int32_t *owner, int64_t nwork,
                            int32_t *oci, double *ov, hipStream_t st) {
    if (n == 0 || nwork == 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_bsr_write_rounds, dim3((unsigned)((nwork + 3) / 4)), dim3(256), 0, st, n,
                       ctb, ccnt, ccols, ctiles, tmx, c, orp, rcnt, rofs, owner, rofs + nb, oci,
                       ov);
    return hipGetLastError();
}

hipError_t bsr_rounds(const int64_t *ccnt, int64_t nb, int64_t *rnd, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_groups, dim3((nb + 255) / 256), dim3(256), 0, st, ccnt, nb, rnd,
                       kWave);
    return hipGetLastError();
}

hipError_t bsr_write(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, const double *tmx, const FilterCtl *c,
                     const int64_t *orp, int32_t *oci, double *ov, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_bsr_write, dim3((nb + 3) / 4), dim3(256), 0, st, n, ctb, ccnt, ccols,
                       ctiles, tmx, c, orp, oci, ov);
    return hipGetLastError();
}

}  // namespace xpm
