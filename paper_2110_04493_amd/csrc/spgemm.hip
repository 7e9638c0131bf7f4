// Sparse-sparse products of the squaring and Taylor steps (Eq. (2.7),
// (4.10), (4.15)) and the masked products of the adjoint, for gfx950.
//
// Row-wise Gustavson, one wavefront per output row, two passes.  The
// symbolic pass marks the output columns of a row in a bit map over
// [lo, hi], the columns the row can reach, and keeps the bit maps.  The
// numeric pass turns a bit map into a perfect hash: the rank of a column
// (prefix popcount) is its slot in the sorted output row, so partial
// products accumulate into a compact LDS array that is already in column
// order and no sort is needed.
//
// Latency is hidden inside the wave rather than by occupancy (long rows need
// tens of KB of LDS each): the left factor's row is read 64 entries at a
// time, one per lane, and broadcast with readlane; a long right-factor row is
// loaded kUnroll chunks of 64 at a time before any LDS work, short ones
// (stencil rows) kShortRows rows at a time, and the accumulation uses LDS
// atomics without return, so nothing waits on them.
// One right-factor row feeds one instruction, so no two lanes of an
// instruction hit the same slot, and the LDS executes a wave's instructions
// in order: the sum for every slot is formed in the left row's storage order
// and the result is bitwise reproducible.
//
// Rows are binned by working-set size; each bin runs with the number of
// waves per block that keeps a block within 64 KB of LDS.  Rows too large for
// LDS run the same code on global scratch (device atomics).
#include <stdlib.h>

#include "kernels.hpp"

namespace xpm {

const int kSymCap[kSymClasses] = {1024, 4096, 16384, 65536, 0};
static const int kSymWpb[kSymClasses] = {8, 8, 4, 1, 4};
const int kNumCap[kNumClasses] = {4096, 8192, 12288, 16384, 24576, 32768, 49152, 65536, 0};
static const int kNumWpb[kNumClasses] = {8, 4, 4, 4, 2, 2, 1, 1, 4};

constexpr int kUnroll = 4;

// Block-to-row mapping of the product kernels.  0 (default): the hardware's
// round-robin over the 8 XCDs, so the whole chip works on one band of
// consecutive rows at a time and the right-factor rows that band reads stay
// in the shared last-level cache.  1: each XCD owns a contiguous slice of
// the rows (better L2 reuse when one slice's working set fits the XCD's L2).
// EXPM_XCD_REMAP=1 in the environment selects 1.
static int g_remap = [] {
    const char *e = getenv("EXPM_XCD_REMAP");
    return e && e[0] == '1' ? 1 : 0;
}();

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <bool kGlobal>
__device__ __forceinline__ void phase_fence() {
    if (kGlobal) __threadfence();
    wave_fence();
}

__device__ __forceinline__ int readlane_i32(int x, int j) {
    return __builtin_amdgcn_readlane(x, j);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t x, int j) {
    int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffff), j);
    int hi = __builtin_amdgcn_readlane((int)(x >> 32), j);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double readlane_f64(double x, int j) {
    return __longlong_as_double(readlane_i64(__double_as_longlong(x), j));
}

// Right-factor rows of at most kShortChunks * 64 entries are loaded
// kShortRows rows at a time (all loads in flight before any LDS work);
// longer rows go one at a time, kUnroll chunks of 64 per round.  Either way
// each call of f covers one chunk of one right-factor row, and the calls
// follow the left row's storage order.
constexpr int kShortRows = 4;
constexpr int kShortChunks = 2;
// Right-factor rows of at most kTinyLen entries (stencil rows) are loaded
// kTinyRows at a time into one 64-lane chunk, kTinyLen lanes per row, and
// then handed to f one row at a time (the lanes of the other rows idle).
constexpr int kTinyRows = 8;
constexpr int kTinyLen = kWave / kTinyRows;

// Values as real (V = double) or complex (V = double2: real and imaginary
// part, interleaved in the value array): load, zero, and the cross-lane
// moves of one value.
template <class V>
__device__ __forceinline__ V load_val(const double *v, int64_t p);
template <>
__device__ __forceinline__ double load_val<double>(const double *v, int64_t p) {
    return v[p];
}
template <>
__device__ __forceinline__ double2 load_val<double2>(const double *v, int64_t p) {
    return ((const double2 *)v)[p];
}
__device__ __forceinline__ double val_readlane(double x, int j) { return readlane_f64(x, j); }
__device__ __forceinline__ double2 val_readlane(double2 x, int j) {
    return make_double2(readlane_f64(x.x, j), readlane_f64(x.y, j));
}
__device__ __forceinline__ double val_shfl(double x, int j) { return __shfl(x, j); }
__device__ __forceinline__ double2 val_shfl(double2 x, int j) {
    return make_double2(__shfl(x.x, j), __shfl(x.y, j));
}
template <class V>
__device__ __forceinline__ V val_zero() {
    return V{};
}

// Calls f(col, a, b) for every partial product a_ik * b_kj of row i of A*B,
// with a_ik taken in A's storage order and, for each of them, B's row k in
// chunks of 64 lanes (f runs on the lanes holding an entry).
template <class V = double, class F>
__device__ __forceinline__ void for_products(const CsrView &A, const CsrView &B, int64_t i,
                                             F &&f) {
    const int lane = lane_id();
    const int64_t b = A.rp[i], e = A.rp[i + 1];
    for (int64_t p0 = b; p0 < e; p0 += kWave) {
        const int64_t p = p0 + lane;
        V av = val_zero<V>();
        int64_t s0 = 0, s1 = 0;
        if (p < e) {
            const int k = A.ci[p];
            av = load_val<V>(A.v, p);
            s0 = B.rp[k];
            s1 = B.rp[k + 1];
        }
        const int m = (int)((e - p0) < kWave ? (e - p0) : kWave);
        const unsigned long long shortm = __ballot(p < e && s1 - s0 <= kShortChunks * kWave);
        const unsigned long long tinym = __ballot(p < e && s1 - s0 <= kTinyLen);
        for (int j = 0; j < m;) {
            {
                const int un = m - j < kTinyRows ? m - j : kTinyRows;
                const unsigned long long grp = ((1ull << un) - 1ull) << j;
                if ((tinym & grp) == grp) {
                    const int u = lane / kTinyLen, h = lane % kTinyLen;
                    const int src = j + (u < un ? u : 0);
                    const int64_t q0 = __shfl(s0, src), q1 = __shfl(s1, src);
                    const V a = val_shfl(av, src);
                    const int64_t q = q0 + h;
                    const bool ok = u < un && q < q1;
                    const int c = ok ? B.ci[q] : -1;
                    const V v = ok ? load_val<V>(B.v, q) : val_zero<V>();
#pragma unroll
                    for (int g = 0; g < kTinyRows; ++g)
                        if (u == g && c >= 0) f(c, a, v);
                    j += un;
                    continue;
                }
            }
            const int un = m - j < kShortRows ? m - j : kShortRows;
            const unsigned long long grp = ((1ull << un) - 1ull) << j;
            if ((shortm & grp) == grp) {
                int c[kShortRows][kShortChunks];
                V v[kShortRows][kShortChunks], a[kShortRows];
#pragma unroll
                for (int u = 0; u < kShortRows; ++u) {
                    const int jj = u < un ? j + u : j;
                    a[u] = val_readlane(av, jj);
                    const int64_t q0 = readlane_i64(s0, jj), q1 = readlane_i64(s1, jj);
#pragma unroll
                    for (int h = 0; h < kShortChunks; ++h) {
                        const int64_t q = q0 + h * kWave + lane;
                        const bool ok = u < un && q < q1;
                        c[u][h] = ok ? B.ci[q] : -1;
                        v[u][h] = ok ? load_val<V>(B.v, q) : val_zero<V>();
                    }
                }
#pragma unroll
                for (int u = 0; u < kShortRows; ++u)
#pragma unroll
                    for (int h = 0; h < kShortChunks; ++h)
                        if (c[u][h] >= 0) f(c[u][h], a[u], v[u][h]);
                j += un;
                continue;
            }
            const V a = val_readlane(av, j);
            const int64_t q0 = readlane_i64(s0, j), q1 = readlane_i64(s1, j);
            for (int64_t qb = q0; qb < q1; qb += kUnroll * kWave) {
                int c[kUnroll];
                V v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t q = qb + u * kWave + lane;
                    c[u] = -1;
                    v[u] = val_zero<V>();
                    if (q < q1) {
                        c[u] = B.ci[q];
                        v[u] = load_val<V>(B.v, q);
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (c[u] >= 0) f(c[u], a, v[u]);
            }
            ++j;
        }
    }
}

// Calls f(col, valid) on every lane for each chunk of 64 entries of the
// right-factor rows that row i of A selects (valid = the lane holds an
// entry).  All lanes take part, so f may use cross-lane operations.  Rows
// of at most kTinyLen entries, eight to a chunk, go instead to g(col), once
// for every lane that holds an entry (g works lane by lane).
template <class F, class G>
__device__ __forceinline__ void for_chunks(const CsrView &A, const CsrView &B, int64_t i, F &&f,
                                           G &&g) {
    const int lane = lane_id();
    const int64_t b = A.rp[i], e = A.rp[i + 1];
    for (int64_t p0 = b; p0 < e; p0 += kWave) {
        const int64_t p = p0 + lane;
        int64_t s0 = 0, s1 = 0;
        if (p < e) {
            const int k = A.ci[p];
            s0 = B.rp[k];
            s1 = B.rp[k + 1];
        }
        const int m = (int)((e - p0) < kWave ? (e - p0) : kWave);
        const unsigned long long shortm = __ballot(p < e && s1 - s0 <= kShortChunks * kWave);
        const unsigned long long tinym = __ballot(p < e && s1 - s0 <= kTinyLen);
        for (int j = 0; j < m;) {
            {
                const int un = m - j < kTinyRows ? m - j : kTinyRows;
                const unsigned long long grp = ((1ull << un) - 1ull) << j;
                if ((tinym & grp) == grp) {
                    const int u = lane / kTinyLen, h = lane % kTinyLen;
                    const int src = j + (u < un ? u : 0);
                    const int64_t q0 = __shfl(s0, src), q1 = __shfl(s1, src);
                    const int64_t q = q0 + h;
                    const int c = u < un && q < q1 ? B.ci[q] : -1;
                    if (c >= 0) g(c);
                    j += un;
                    continue;
                }
            }
            const int un = m - j < kShortRows ? m - j : kShortRows;
            const unsigned long long grp = ((1ull << un) - 1ull) << j;
            if ((shortm & grp) == grp) {
                int c[kShortRows][kShortChunks];
                bool any[kShortRows][kShortChunks];
#pragma unroll
                for (int u = 0; u < kShortRows; ++u) {
                    const int jj = u < un ? j + u : j;
                    const int64_t q0 = readlane_i64(s0, jj), q1 = readlane_i64(s1, jj);
#pragma unroll
                    for (int h = 0; h < kShortChunks; ++h) {
                        const int64_t q = q0 + h * kWave + lane;
                        c[u][h] = u < un && q < q1 ? B.ci[q] : -1;
                        any[u][h] = u < un && q0 + h * kWave < q1;   // uniform
                    }
                }
#pragma unroll
                for (int u = 0; u < kShortRows; ++u)
#pragma unroll
                    for (int h = 0; h < kShortChunks; ++h)
                        if (any[u][h]) f(c[u][h], c[u][h] >= 0);
                j += un;
                continue;
            }
            const int64_t q0 = readlane_i64(s0, j), q1 = readlane_i64(s1, j);
            for (int64_t qb = q0; qb < q1; qb += kUnroll * kWave) {
                int c[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t q = qb + u * kWave + lane;
                    c[u] = q < q1 ? B.ci[q] : -1;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (qb + u * kWave < q1) f(c[u], c[u] >= 0);
            }
            ++j;
        }
    }
}

// ============================================================== binning
// kind 0: symbolic (bit map), 1: numeric and masked (accumulator + bit map
// with prefix counts), 2: numeric on complex values (two accumulators per
// slot).
__device__ __forceinline__ int64_t row_bytes(int kind, int64_t W, int64_t c) {
    return kind == 0 ? 4 * W : (kind == 2 ? 16 : 8) * c + 8 * W;
}

struct Caps {
    int cap[12];
    int ncls;
};

static Caps make_caps(int kind) {
    Caps caps;
    caps.ncls = kind == 0 ? kSymClasses : kNumClasses;
    for (int j = 0; j < caps.ncls; j++) caps.cap[j] = kind == 0 ? kSymCap[j] : kNumCap[j];
    return caps;
}

// Appends row i to its class list.  All lanes of the wave call it (valid =
// the lane has a row); the lanes of one class share a single atomic, so the
// handful of class counters see one update per class per wave.
__device__ __forceinline__ void bin_one(int64_t i, bool valid, int64_t n, int64_t bytes,
                                        const Caps &caps, int *counts, int32_t *lists) {
    int cls = caps.ncls - 1;
    for (int j = 0; j < caps.ncls - 1; j++)
        if (bytes <= caps.cap[j]) {
            cls = j;
            break;
        }
    if (!valid) cls = -1;
    const unsigned long long lt = (1ull << lane_id()) - 1ull;
    for (int c = 0; c < caps.ncls; ++c) {
        const unsigned long long m = __ballot(cls == c);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&counts[c], __popcll(m));
        base = __shfl(base, leader);
        if (cls == c) lists[(int64_t)c * n + base + __popcll(m & lt)] = (int32_t)i;
    }
}

__global__ void k_bin(const int64_t *woff, const int64_t *crp, int64_t n, int kind, Caps caps,
                      int *counts, int32_t *lists) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    int64_t bytes = 0;
    if (valid) {
        const int64_t W = woff[i + 1] - woff[i];
        const int64_t c = crp ? crp[i + 1] - crp[i] : 0;
        bytes = row_bytes(kind, W, c);
    }
    bin_one(i, valid, n, bytes, caps, counts, lists);
}

hipError_t bin_rows(const int64_t *woff, const int64_t *crp, int64_t n, int kind, int *counts,
                    int32_t *lists, hipStream_t st) {
    Caps caps = make_caps(kind);
    hipError_t e = hipMemsetAsync(counts, 0, sizeof(int) * caps.ncls, st);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3((n + 255) / 256), dim3(256), 0, st, woff, crp, n, kind, caps,
                       counts, lists);
    return hipGetLastError();
}

// ============================================================== row bounds

__global__ void k_row_bounds(CsrView A, CsrView B, int addA, int32_t *lo, int64_t *words,
                             int64_t *ub) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= A.n) return;
    int mn = INT32_MAX, mx = -1;
    long long s = 0;
    int64_t b = A.rp[i], e = A.rp[i + 1];
    for (int64_t p = b + lane_id(); p < e; p += kWave) {
        int k = A.ci[p];
        int64_t q0 = B.rp[k], q1 = B.rp[k + 1];
        if (q1 > q0) {
            mn = min(mn, B.ci[q0]);
            mx = max(mx, B.ci[q1 - 1]);
            s += q1 - q0;
        }
    }
    if (addA && e > b && lane_id() == 0) {
        mn = min(mn, A.ci[b]);
        mx = max(mx, A.ci[e - 1]);
        s += e - b;
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    s = wave_sum_ll(s);
    if (lane_id() == 0) {
        if (mx < 0) {
            lo[i] = 0;
            words[i] = 0;
        } else {
            int l = mn & ~31;
            lo[i] = l;
            words[i] = ((mx - l) >> 5) + 1;
        }
        ub[i] = s;
    }
}

hipError_t row_bounds(CsrView A, CsrView B, int addA, int32_t *lo, int64_t *words, int64_t *ub,
                      hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    int wpb = 4;
    hipLaunchKernelGGL(k_row_bounds, dim3((A.n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, A, B,
                       addA, lo, words, ub);
    return hipGetLastError();
}

// ============================================================== symbolic

template <bool kGlobal>
__global__ __launch_bounds__(512) void k_symbolic(CsrView A, CsrView B, int addA,
                                                  const int32_t *__restrict__ lo,
                                                  const int64_t *__restrict__ woff,
                                                  uint32_t *__restrict__ bitmaps,
                                                  int64_t *__restrict__ cnt,
                                                  const int32_t *__restrict__ list, int nlist,
                                                  int wpb, int remap, int cap_words) {
    extern __shared__ uint32_t smem_u32[];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int64_t idx = (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * wpb + wave;
    if (idx >= nlist) return;
    const int64_t i = list[idx];
    const int64_t w0 = woff[i], W = woff[i + 1] - w0;
    if (W == 0) {
        if (lane == 0) cnt[i] = 0;
        return;
    }
    uint32_t *bm = kGlobal ? bitmaps + w0 : smem_u32 + (int64_t)wave * cap_words;
    for (int64_t w = lane; w < W; w += kWave) bm[w] = 0;
    phase_fence<kGlobal>();
    const int base = lo[i];
    if (addA) {
        for (int64_t p = A.rp[i] + lane; p < A.rp[i + 1]; p += kWave) {
            const int d = A.ci[p] - base;
            atomicOr(&bm[d >> 5], 1u << (d & 31));
        }
    }
    for_chunks(A, B, i, [&](int col, bool valid) {
        // The columns of one chunk are sorted, so the lanes that share a
        // bit-map word form contiguous segments.  A segment of consecutive
        // columns (the common case for banded and grid-like rows) is set by
        // its first lane with one atomic; other segments set bit by bit.
        const int d = valid ? col - base : 0;
        const int w = valid ? (d >> 5) : -1 - lane;   // invalid lanes: own segment
        const int wprev = __shfl_up(w, 1);
        const bool head = lane == 0 || wprev != w;
        const unsigned long long heads = __ballot(head);
        const int h = 63 - __clzll(heads & ((2ull << lane) - 1ull));    // my segment's head
        const unsigned long long nxt = h == 63 ? 0ull : heads & ~((2ull << h) - 1ull);
        const int end = nxt ? __ffsll((long long)nxt) - 2 : 63;         // its last lane
        const int dfirst = __shfl(d, h), dlast = __shfl(d, end);
        if (!valid) return;
        if (dlast - dfirst == end - h) {
            if (lane == h) {
                const int b0 = dfirst & 31, b1 = dlast & 31;
                const unsigned hi = b1 == 31 ? ~0u : ((2u << b1) - 1u);
                atomicOr(&bm[w], hi & ~((1u << b0) - 1u));
            }
        } else {
            atomicOr(&bm[w], 1u << (d & 31));
        }
    }, [&](int col) {
        const int d = col - base;
        atomicOr(&bm[d >> 5], 1u << (d & 31));
    });
    phase_fence<kGlobal>();
    long long s = 0;
    for (int64_t w = lane; w < W; w += kWave) {
        const uint32_t x = bm[w];
        s += __popc(x);
        if (!kGlobal) bitmaps[w0 + w] = x;
    }
    s = wave_sum_ll(s);
    if (lane == 0) cnt[i] = s;
}

hipError_t symbolic(CsrView A, CsrView B, int addA, const int32_t *lo, const int64_t *woff,
                    uint32_t *bitmaps, int64_t *cnt, const int *host_counts,
                    const int32_t *lists, int64_t n, hipStream_t st) {
    for (int c = 0; c < kSymClasses; c++) {
        const int m = host_counts[c];
        if (m == 0) continue;
        const int wpb = kSymWpb[c];
        dim3 grid((m + wpb - 1) / wpb), block(wpb * kWave);
        const int32_t *list = lists + (int64_t)c * n;
        if (kSymCap[c] > 0)
            hipLaunchKernelGGL(k_symbolic<false>, grid, block, (size_t)wpb * kSymCap[c], st, A, B,
                               addA, lo, woff, bitmaps, cnt, list, m, wpb, g_remap, kSymCap[c] / 4);
        else
            hipLaunchKernelGGL(k_symbolic<true>, grid, block, 0, st, A, B, addA, lo, woff,
                               bitmaps, cnt, list, m, wpb, g_remap, 0);
    }
    return hipGetLastError();
}

// ============================================================== rank tables

// (bit-map word, exclusive popcount prefix) pairs of one row.
__device__ __forceinline__ void load_rank_table(const uint32_t *__restrict__ src, int64_t W,
                                                uint2 *bp) {
    unsigned carry = 0;
    for (int64_t w0 = 0; w0 < W; w0 += kWave) {
        const int64_t w = w0 + lane_id();
        const uint32_t x = w < W ? src[w] : 0u;
        const unsigned pc = __popc(x);
        const unsigned inc = wave_incl_scan(pc);
        if (w < W) bp[w] = make_uint2(x, carry + inc - pc);
        carry += __shfl(inc, kWave - 1);
    }
}

__device__ __forceinline__ unsigned rank_of(const uint2 *bp, int d) {
    const uint2 e = bp[d >> 5];
    return e.y + __popc(e.x & ((1u << (d & 31)) - 1u));
}

// Column of the t-th set bit of the rank table (binary search on the prefix
// counts, then selection inside the word).
__device__ __forceinline__ int column_of(const uint2 *bp, int64_t W, unsigned t, int base) {
    int64_t lo = 0, hi = W - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (bp[mid].y <= t) lo = mid; else hi = mid - 1;
    }
    const uint2 e = bp[lo];
    uint32_t x = e.x;
    for (unsigned r = t - e.y; r > 0; --r) x &= x - 1;
    return base + 32 * (int)lo + (__ffs(x) - 1);
}

template <bool kGlobal>
__device__ __forceinline__ void acc_add(double *p, double x) {
    atomicAdd(p, x);
}

// ============================================================== numeric

template <bool kGlobal>
__global__ __launch_bounds__(512) void k_numeric(
    CsrView A, CsrView B, double alphaA, double div, const int32_t *__restrict__ lo,
    const int64_t *__restrict__ woff, const uint32_t *__restrict__ bitmaps,
    const int64_t *__restrict__ crp, int32_t *__restrict__ cci, double *__restrict__ cv,
    double *__restrict__ rowsq, const int32_t *__restrict__ list, int nlist, int wpb,
    int remap, int cap_bytes, char *__restrict__ scratch,
    const int64_t *__restrict__ scratch_off) {
    extern __shared__ double smem_f64[];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int64_t idx = (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * wpb + wave;
    if (idx >= nlist) return;
    const int64_t i = list[idx];
    const int64_t w0 = woff[i], W = woff[i + 1] - w0;
    const int64_t o = crp[i], c = crp[i + 1] - o;
    if (c == 0) {
        if (rowsq && lane == 0) rowsq[i] = 1.0;
        return;
    }
    char *mem = kGlobal ? scratch + scratch_off[i] : (char *)smem_f64 + (int64_t)wave * cap_bytes;
    double *acc = (double *)mem;
    uint2 *bp = (uint2 *)(mem + 8 * c);
    const int base = lo[i];

    load_rank_table(bitmaps + w0, W, bp);
    for (int64_t t = lane; t < c; t += kWave) acc[t] = 0.0;
    phase_fence<kGlobal>();
    if (alphaA != 0.0) {
        for (int64_t p = A.rp[i] + lane; p < A.rp[i + 1]; p += kWave)
            acc_add<kGlobal>(&acc[rank_of(bp, A.ci[p] - base)], alphaA * A.v[p]);
    }
    for_products(A, B, i, [&](int col, double a, double bv) {
        acc_add<kGlobal>(&acc[rank_of(bp, col - base)], a * bv);
    });
    phase_fence<kGlobal>();
    double s = 0.0;
    bool diag = false;
    for (int64_t t = lane; t < c; t += kWave) {
        const int col = column_of(bp, W, (unsigned)t, base);
        double val = acc[t];
        if (div != 1.0) val = val / div;
        cci[o + t] = col;
        cv[o + t] = val;
        if (rowsq) {
            const double f = col == i ? val + 1.0 : val;
            diag |= col == i;
            s = fma(f, f, s);
        }
    }
    if (rowsq) {
        s = wave_sum(s);
        const bool any = __ballot(diag) != 0;
        if (lane == 0) rowsq[i] = any ? s : s + 1.0;
    }
}

__global__ void k_numeric_scratch(const int64_t *woff, const int64_t *crp, int64_t n,
                                  int kind, int64_t *bytes) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t need = row_bytes(kind, woff[i + 1] - woff[i], crp[i + 1] - crp[i]);
    bytes[i] = need <= kNumCap[kNumClasses - 2] ? 0 : (need + 255) & ~int64_t(255);
}

hipError_t numeric_scratch_sizes(const int64_t *woff, const int64_t *crp, int64_t n,
                                 int64_t *bytes, hipStream_t st, bool cplx) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_numeric_scratch, dim3((n + 255) / 256), dim3(256), 0, st, woff, crp, n,
                       cplx ? 2 : 1, bytes);
    return hipGetLastError();
}

hipError_t numeric(CsrView A, CsrView B, double alphaA, double div, const int32_t *lo,
                   const int64_t *woff, const uint32_t *bitmaps, const int64_t *crp, int32_t *cci,
                   double *cv, double *rowsq, const int *host_counts, const int32_t *lists,
                   int64_t n, void *scratch, const int64_t *scratch_off, hipStream_t st) {
    for (int c = 0; c < kNumClasses; c++) {
        const int m = host_counts[c];
        if (m == 0) continue;
        const int wpb = kNumWpb[c];
        dim3 grid((m + wpb - 1) / wpb), block(wpb * kWave);
        const int32_t *list = lists + (int64_t)c * n;
        if (kNumCap[c] > 0)
            hipLaunchKernelGGL(k_numeric<false>, grid, block, (size_t)wpb * kNumCap[c], st, A, B,
                               alphaA, div, lo, woff, bitmaps, crp, cci, cv, rowsq, list, m, wpb,
                               g_remap, kNumCap[c], (char *)nullptr, (const int64_t *)nullptr);
        else
            hipLaunchKernelGGL(k_numeric<true>, grid, block, 0, st, A, B, alphaA, div, lo, woff,
                               bitmaps, crp, cci, cv, rowsq, list, m, wpb, g_remap, 0, (char *)scratch,
                               scratch_off);
    }
    return hipGetLastError();
}

// Complex values (a double2 per entry, real and imaginary part): the same
// product with two LDS accumulators per slot, added one after the other in
// the same order as the real kernel's single one.
template <bool kGlobal>
__global__ __launch_bounds__(512) void k_numeric_z(
    CsrView A, CsrView B, double alphaA, double div, const int32_t *__restrict__ lo,
    const int64_t *__restrict__ woff, const uint32_t *__restrict__ bitmaps,
    const int64_t *__restrict__ crp, int32_t *__restrict__ cci, double2 *__restrict__ cv,
    double *__restrict__ rowsq, const int32_t *__restrict__ list, int nlist, int wpb,
    int remap, int cap_bytes, char *__restrict__ scratch,
    const int64_t *__restrict__ scratch_off) {
    extern __shared__ double smem_f64[];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int64_t idx = (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * wpb + wave;
    if (idx >= nlist) return;
    const int64_t i = list[idx];
    const int64_t w0 = woff[i], W = woff[i + 1] - w0;
    const int64_t o = crp[i], c = crp[i + 1] - o;
    if (c == 0) {
        if (rowsq && lane == 0) rowsq[i] = 1.0;
        return;
    }
    char *mem = kGlobal ? scratch + scratch_off[i] : (char *)smem_f64 + (int64_t)wave * cap_bytes;
    double *acc = (double *)mem;   // slot t: acc[2t] real, acc[2t + 1] imaginary part
    uint2 *bp = (uint2 *)(mem + 16 * c);
    const int base = lo[i];

    load_rank_table(bitmaps + w0, W, bp);
    for (int64_t t = lane; t < 2 * c; t += kWave) acc[t] = 0.0;
    phase_fence<kGlobal>();
    if (alphaA != 0.0) {
        for (int64_t p = A.rp[i] + lane; p < A.rp[i + 1]; p += kWave) {
            const unsigned r = rank_of(bp, A.ci[p] - base);
            const double2 z = load_val<double2>(A.v, p);
            acc_add<kGlobal>(&acc[2 * r], alphaA * z.x);
            acc_add<kGlobal>(&acc[2 * r + 1], alphaA * z.y);
        }
    }
    for_products<double2>(A, B, i, [&](int col, double2 a, double2 bv) {
        const unsigned r = rank_of(bp, col - base);
        acc_add<kGlobal>(&acc[2 * r], a.x * bv.x - a.y * bv.y);
        acc_add<kGlobal>(&acc[2 * r + 1], a.x * bv.y + a.y * bv.x);
    });
    phase_fence<kGlobal>();
    double s = 0.0;
    bool diag = false;
    for (int64_t t = lane; t < c; t += kWave) {
        const int col = column_of(bp, W, (unsigned)t, base);
        double re = acc[2 * t], im = acc[2 * t + 1];
        if (div != 1.0) {
            re = re / div;
            im = im / div;
        }
        cci[o + t] = col;
        cv[o + t] = make_double2(re, im);
        if (rowsq) {
            const double f = col == i ? re + 1.0 : re;
            diag |= col == i;
            s = fma(f, f, s);
            s = fma(im, im, s);
        }
    }
    if (rowsq) {
        s = wave_sum(s);
        const bool any = __ballot(diag) != 0;
        if (lane == 0) rowsq[i] = any ? s : s + 1.0;
    }
}

hipError_t numeric_z(CsrView A, CsrView B, double alphaA, double div, const int32_t *lo,
                     const int64_t *woff, const uint32_t *bitmaps, const int64_t *crp,
                     int32_t *cci, double *cv, double *rowsq, const int *host_counts,
                     const int32_t *lists, int64_t n, void *scratch, const int64_t *scratch_off,
                     hipStream_t st) {
    for (int c = 0; c < kNumClasses; c++) {
        const int m = host_counts[c];
        if (m == 0) continue;
        const int wpb = kNumWpb[c];
        dim3 grid((m + wpb - 1) / wpb), block(wpb * kWave);
        const int32_t *list = lists + (int64_t)c * n;
        if (kNumCap[c] > 0)
            hipLaunchKernelGGL(k_numeric_z<false>, grid, block, (size_t)wpb * kNumCap[c], st, A,
                               B, alphaA, div, lo, woff, bitmaps, crp, cci, (double2 *)cv, rowsq,
                               list, m, wpb, g_remap, kNumCap[c], (char *)nullptr,
                               (const int64_t *)nullptr);
        else
            hipLaunchKernelGGL(k_numeric_z<true>, grid, block, 0, st, A, B, alphaA, div, lo, woff,
                               bitmaps, crp, cci, (double2 *)cv, rowsq, list, m, wpb, g_remap, 0,
                               (char *)scratch, scratch_off);
    }
    return hipGetLastError();
}

// ============================================================== masked products
// One wave per mask row; the mask row's columns form the rank table and
// partial products whose column is not in the mask are skipped.

template <bool kGlobal>
__global__ __launch_bounds__(512) void k_masked(
    CsrView M, CsrView D, double gamma, MaskTerm t1, MaskTerm t2, double div,
    double *__restrict__ out, const int32_t *__restrict__ list, int nlist, int wpb,
    int remap, int cap_bytes, char *__restrict__ scratch,
    const int64_t *__restrict__ scratch_off) {
    extern __shared__ double smem_f64[];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int64_t idx = (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * wpb + wave;
    if (idx >= nlist) return;
    const int64_t i = list[idx];
    const int64_t o = M.rp[i], c = M.rp[i + 1] - o;
    if (c == 0) return;
    const int lo = M.ci[o] & ~31;
    const int64_t W = ((M.ci[o + c - 1] - lo) >> 5) + 1;
    char *mem = kGlobal ? scratch + scratch_off[i] : (char *)smem_f64 + (int64_t)wave * cap_bytes;
    double *acc = (double *)mem;
    uint2 *bp = (uint2 *)(mem + 8 * c);
    for (int64_t w = lane; w < W; w += kWave) bp[w] = make_uint2(0u, 0u);
    for (int64_t t = lane; t < c; t += kWave) acc[t] = 0.0;
    phase_fence<kGlobal>();
    for (int64_t t = lane; t < c; t += kWave) {
        const int d = M.ci[o + t] - lo;
        atomicOr(&bp[d >> 5].x, 1u << (d & 31));
    }
    phase_fence<kGlobal>();
    {   // prefix counts
        unsigned carry = 0;
        for (int64_t w0 = 0; w0 < W; w0 += kWave) {
            const int64_t w = w0 + lane;
            const uint32_t x = w < W ? bp[w].x : 0u;
            const unsigned pc = __popc(x);
            const unsigned inc = wave_incl_scan(pc);
            if (w < W) bp[w].y = carry + inc - pc;
            carry += __shfl(inc, kWave - 1);
        }
    }
    phase_fence<kGlobal>();
    const int hi = lo + 32 * (int)W;
    auto add_masked = [&](int col, double x) {
        if (col < lo || col >= hi) return;
        const int d = col - lo;
        const uint2 e2 = bp[d >> 5];
        const unsigned bit = 1u << (d & 31);
        if (!(e2.x & bit)) return;
        acc_add<kGlobal>(&acc[e2.y + __popc(e2.x & (bit - 1u))], x);
    };
    if (t1.A.n != 0 && t1.alpha != 0.0) {
        const double al = t1.alpha;
        for_products(t1.A, t1.B, i, [&](int col, double a, double bv) {
            add_masked(col, (al * a) * bv);
        });
    }
    if (t2.A.n != 0 && t2.alpha != 0.0) {
        const double al = t2.alpha;
        for_products(t2.A, t2.B, i, [&](int col, double a, double bv) {
            add_masked(col, (al * a) * bv);
        });
    }
    phase_fence<kGlobal>();
    if (div != 1.0) {
        for (int64_t t = lane; t < c; t += kWave) acc[t] = acc[t] / div;
        phase_fence<kGlobal>();
    }
    if (D.n != 0 && gamma != 0.0) {
        for (int64_t p = D.rp[i] + lane; p < D.rp[i + 1]; p += kWave)
            add_masked(D.ci[p], gamma * D.v[p]);
        phase_fence<kGlobal>();
    }
    for (int64_t t = lane; t < c; t += kWave) out[o + t] = acc[t];
}

// Inner-product form of a single masked product: one wave per row r of M.
// A's row r (its column keys and values) is staged in LDS, and each entry of
// B's column c is looked up among A's keys by binary search.  When the mask
// row has at most kDotCols entries whose B columns hold at most
// kDotChunks * 64 entries together, all of them are loaded at once (their
// keys and positions, then their values: two memory round trips for the
// whole row), the products go to LDS and each output sums its own span of
// them in a fixed order.  Other rows take the columns one at a time, each
// lane accumulating its own products before a fixed butterfly adds the
// lanes.  Either way the result is reproducible.  Rows of A longer than the
// LDS stage are searched in memory.
constexpr int kDotWaves = 4, kDotLds = 512;
constexpr int kDotCols = 8, kDotChunks = 8;

__global__ __launch_bounds__(kWave * kDotWaves) void k_masked_dot(
    CsrView M, const double *__restrict__ dv, PosCsr A, PosCsr Bt, double div,
    double *__restrict__ out) {
    __shared__ int32_t skey[kDotWaves][kDotLds];
    __shared__ double sval[kDotWaves][kDotLds];
    __shared__ double sprod[kDotWaves][kDotChunks * kWave];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * kDotWaves + wv;
    if (r >= M.n) return;
    const int64_t mo = M.rp[r], ml = M.rp[r + 1] - mo;
    if (ml == 0) return;
    const int64_t ao = A.rp[r], al = A.rp[r + 1] - ao;
    const bool staged = al <= kDotLds;
    int32_t *key = skey[wv];
    double *val = sval[wv];
    if (staged) {
        for (int64_t t = lane; t < al; t += kWave) {
            key[t] = A.ci[ao + t];
            val[t] = A.v[A.pos[ao + t]];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // the position of key k among A's row r, or -1
    auto find = [&](int32_t k) -> int64_t {
        int64_t lo = 0, hi = al;
        if (staged) {
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (key[mid] < k) lo = mid + 1; else hi = mid;
            }
            return lo < al && key[lo] == k ? lo : -1;
        }
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (A.ci[ao + mid] < k) lo = mid + 1; else hi = mid;
        }
        return lo < al && A.ci[ao + lo] == k ? lo : -1;
    };
    auto a_at = [&](int64_t j) { return staged ? val[j] : A.v[A.pos[ao + j]]; };
    if (staged && ml <= kDotCols) {
        int64_t b0 = 0, len = 0;
        if (lane < ml) {
            const int32_t c = M.ci[mo + lane];
            b0 = Bt.rp[c];
            len = Bt.rp[c + 1] - b0;
        }
        int64_t st[kDotCols + 1], bs[kDotCols];
        st[0] = 0;
#pragma unroll
        for (int t = 0; t < kDotCols; ++t) {
            bs[t] = t < ml ? readlane_i64(b0, t) : 0;
            st[t + 1] = st[t] + (t < ml ? readlane_i64(len, t) : 0);
        }
        const int64_t tot = st[kDotCols];
        if (tot <= kDotChunks * kWave) {
            double *prod = sprod[wv];
            int32_t kq[kDotChunks];
            int64_t pq[kDotChunks];
            double vq[kDotChunks];
#pragma unroll
            for (int q = 0; q < kDotChunks; ++q) {
                const int64_t f = q * kWave + lane;
                int t = 0;
#pragma unroll
                for (int u = 1; u < kDotCols; ++u)
                    if (u < ml && f >= st[u]) t = u;
                const bool ok = f < tot;
                const int64_t p = bs[t] + (f - st[t]);
                kq[q] = ok ? Bt.ci[p] : -1;
                pq[q] = ok ? Bt.pos[p] : 0;
            }
#pragma unroll
            for (int q = 0; q < kDotChunks; ++q) vq[q] = kq[q] >= 0 ? Bt.v[pq[q]] : 0.0;
#pragma unroll
            for (int q = 0; q < kDotChunks; ++q) {
                const int64_t f = q * kWave + lane;
                if (f < tot) {
                    const int64_t j = find(kq[q]);
                    prod[f] = j >= 0 ? val[j] * vq[q] : 0.0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int t = 0; t < kDotCols; ++t) {
                if (t >= ml) break;
                double s = 0.0;
                for (int64_t f = st[t] + lane; f < st[t + 1]; f += kWave) s += prod[f];
                s = wave_sum(s);
                if (lane == 0) out[mo + t] = s / div + dv[mo + t];
            }
            return;
        }
    }
    for (int64_t t = 0; t < ml; ++t) {
        const int32_t c = M.ci[mo + t];
        double s = 0.0;
        if (al > 0) {
            for (int64_t p = Bt.rp[c] + lane; p < Bt.rp[c + 1]; p += kWave) {
                const int64_t j = find(Bt.ci[p]);
                if (j >= 0) s += a_at(j) * Bt.v[Bt.pos[p]];
            }
        }
        s = wave_sum(s);
        if (lane == 0) out[mo + t] = s / div + dv[mo + t];
    }
}

hipError_t masked_dot(CsrView M, const double *dv, PosCsr A, PosCsr Bt, double div, double *out,
                      hipStream_t st) {
    if (M.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_masked_dot, dim3((unsigned)((M.n + kDotWaves - 1) / kDotWaves)),
                       dim3(kWave * kDotWaves), 0, st, M, dv, A, Bt, div, out);
    return hipGetLastError();
}

__global__ void k_masked_bin(CsrView M, Caps caps, int *counts, int32_t *lists, int64_t *sb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < M.n;
    int64_t bytes = 0;
    if (valid) {
        const int64_t o = M.rp[i], c = M.rp[i + 1] - o;
        const int64_t W = c ? ((M.ci[o + c - 1] - (M.ci[o] & ~31)) >> 5) + 1 : 0;
        bytes = row_bytes(1, W, c);
    }
    bin_one(i, valid, M.n, bytes, caps, counts, lists);
    if (valid) sb[i] = bytes <= kNumCap[kNumClasses - 2] ? 0 : (bytes + 255) & ~int64_t(255);
}

// scratch layout: sb[n+1] int64 | off[n+1] int64 | counts[16] int |
// lists[kNumClasses*n] int32 | scan tmp | global rows' memory
size_t masked_meta_bytes(int64_t n) {
    size_t b = sizeof(int64_t) * (2 * (size_t)n + 2) + 16 * sizeof(int) +
               sizeof(int32_t) * (size_t)kNumClasses * n;
    b = (b + 255) & ~(size_t)255;
    b += (scan_tmp_bytes(n) + 255) & ~(size_t)255;
    return b + 256;
}

hipError_t masked_products(CsrView M, CsrView D, double gamma, MaskTerm t1, MaskTerm t2,
                           double div, double *out, void *scratch, size_t scratch_bytes,
                           size_t *needed, hipStream_t st) {
    const int64_t n = M.n;
    if (n == 0) return hipSuccess;
    if (masked_meta_bytes(n) > scratch_bytes) {
        if (needed) *needed = masked_meta_bytes(n);
        return hipErrorOutOfMemory;
    }
    char *s = (char *)scratch;
    int64_t *sb = (int64_t *)s;
    int64_t *off = sb + n + 1;
    int *counts = (int *)(off + n + 1);
    int32_t *lists = (int32_t *)(counts + 16);
    char *scan_tmp = (char *)(lists + (int64_t)kNumClasses * n);
    scan_tmp = (char *)(((uintptr_t)scan_tmp + 255) & ~(uintptr_t)255);
    char *glob = scan_tmp + ((scan_tmp_bytes(n) + 255) & ~(size_t)255);
    const size_t used = (size_t)(glob - s);
    Caps caps = make_caps(1);
    hipError_t e = hipMemsetAsync(counts, 0, sizeof(int) * 16, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_masked_bin, dim3((n + 255) / 256), dim3(256), 0, st, M, caps, counts,
                       lists, sb);
    e = scan_i64(sb, off, n, scan_tmp, scan_tmp_bytes(n), st);
    if (e != hipSuccess) return e;
    int hc[16];
    int64_t gbytes = 0;
    e = hipMemcpyAsync(hc, counts, sizeof(int) * kNumClasses, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&gbytes, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (needed) *needed = used + (size_t)gbytes;
    if (used + (size_t)gbytes > scratch_bytes) return hipErrorOutOfMemory;
    for (int c = 0; c < kNumClasses; c++) {
        const int m = hc[c];
        if (m == 0) continue;
        const int wpb = kNumWpb[c];
        dim3 grid((m + wpb - 1) / wpb), block(wpb * kWave);
        const int32_t *list = lists + (int64_t)c * n;
        if (kNumCap[c] > 0)
            hipLaunchKernelGGL(k_masked<false>, grid, block, (size_t)wpb * kNumCap[c], st, M, D,
                               gamma, t1, t2, div, out, list, m, wpb, g_remap, kNumCap[c],
                               (char *)nullptr,
                               (const int64_t *)nullptr);
        else
            hipLaunchKernelGGL(k_masked<true>, grid, block, 0, st, M, D, gamma, t1, t2, div, out,
                               list, m, wpb, g_remap, 0, glob, off);
    }
    return hipGetLastError();
}

}  // namespace xpm
