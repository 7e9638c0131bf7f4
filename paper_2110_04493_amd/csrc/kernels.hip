// gfx950 kernels of the filtered precise-integration sparse exponential:
// scans, reductions, checks, the device side of Algorithm 4.1 (filter
// passes and controller), compaction with the identity insert of
// Algorithm 4.2 step 5, sparse addition and transposition.  The sparse
// products themselves are in spgemm.hip.
#include "kernels.hpp"

#include <math.h>

#include <type_traits>

namespace xpm {

// ============================================================== scan
// Three-phase exclusive scan: per-block sums, a scan of the block sums in
// one block, then the block-local scans with their offsets.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ long long block_excl_scan(long long x, long long *total) {
    __shared__ long long ws[kScanBlock / kWave];
    long long inc = wave_incl_scan_ll(x);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) ws[w] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
    for (int j = 0; j < kScanBlock / kWave; j++) {
        if (j < w) off += ws[j];
        tot += ws[j];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int64_t *in, int64_t n,
                                                            int64_t *bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    long long s = 0;
    for (int j = 0; j < kScanItems; j++) {
        int64_t idx = base + (int64_t)j * kScanBlock + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    long long tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocksums(int64_t *bsum, int64_t nb,
                                                               int64_t *total_out) {
    long long carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        int64_t idx = base + threadIdx.x;
        long long x = idx < nb ? bsum[idx] : 0;
        long long tot;
        long long ex = block_excl_scan(x, &tot);
        if (idx < nb) bsum[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const int64_t *in, int64_t n,
                                                           const int64_t *bsum, int64_t *out) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long s = 0;
    for (int j = 0; j < kScanItems; j++) {
        int64_t idx = base + j;
        v[j] = idx < n ? in[idx] : 0;
        s += v[j];
    }
    long long tot;
    long long ex = block_excl_scan(s, &tot) + bsum[blockIdx.x];
    for (int j = 0; j < kScanItems; j++) {
        int64_t idx = base + j;
        if (idx < n) out[idx] = ex;
        ex += v[j];
    }
}

// k_scan_final with each block's offset summed by the block itself from the
// reduce pass's block totals (for few blocks: one launch fewer than a
// separate pass over them); the last block writes the total to out[n].
constexpr int64_t kScanFuseBlocks = 2048;

__global__ __launch_bounds__(kScanBlock) void k_scan_final_fused(const int64_t *in, int64_t n,
                                                                 const int64_t *bsum, int64_t nb,
                                                                 int64_t *out) {
    long long part = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kScanBlock) part += bsum[b];
    long long boff;
    block_excl_scan(part, &boff);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long s = 0;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t idx = base + j;
        v[j] = idx < n ? in[idx] : 0;
        s += v[j];
    }
    long long tot;
    long long ex = block_excl_scan(s, &tot) + boff;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t idx = base + j;
        if (idx < n) out[idx] = ex;
        ex += v[j];
    }
    if ((int64_t)blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = boff + tot;
}

// Arrays of up to kScanSmall entries are scanned by one block in one launch
// (tile by tile with a running carry): most scans here are over block rows
// or panels, where the three launches would cost more than the work.
constexpr int64_t kScanSmall = 16 * kScanTile;

__global__ __launch_bounds__(kScanBlock) void k_scan_one(const int64_t *in, int64_t n,
                                                         int64_t *out) {
    long long carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kScanTile) {
        const int64_t base = t0 + (int64_t)threadIdx.x * kScanItems;
        long long v[kScanItems];
        long long s = 0;
        for (int j = 0; j < kScanItems; j++) {
            const int64_t idx = base + j;
            v[j] = idx < n ? in[idx] : 0;
            s += v[j];
        }
        long long tot;
        long long ex = block_excl_scan(s, &tot) + carry;
        for (int j = 0; j < kScanItems; j++) {
            const int64_t idx = base + j;
            if (idx < n) out[idx] = ex;
            ex += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

size_t scan_tmp_bytes(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

hipError_t scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes,
                    hipStream_t st) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (tmp_bytes < scan_tmp_bytes(n)) return hipErrorInvalidValue;
    int64_t *bsum = (int64_t *)tmp;
    if (n == 0) {
        return hipMemsetAsync(out, 0, sizeof(int64_t), st);
    }
    if (n <= kScanSmall) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanBlock), 0, st, in, n, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, st, in, n, bsum);
    if (nb <= kScanFuseBlocks) {
        hipLaunchKernelGGL(k_scan_final_fused, dim3(nb), dim3(kScanBlock), 0, st, in, n, bsum,
                           nb, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(kScanBlock), 0, st, bsum, nb, out + n);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanBlock), 0, st, in, n, bsum, out);
    return hipGetLastError();
}

// ============================================================== checks, norms

__global__ void k_validate(CsrView A, int64_t nnz, int *flag) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= A.n) return;
    int f = 0;
    int64_t b = A.rp[i], e = A.rp[i + 1];
    // every row checks both of its bounds: rows run in parallel, so a row
    // cannot rely on the previous row's check of its start
    if (i == 0 && b != 0) f |= 1;
    if (b < 0 || b > nnz || e < b || e > nnz) f |= 1;
    if (!(f & 1)) {
        for (int64_t p = b + lane_id(); p < e; p += kWave) {
            int c = A.ci[p];
            if (c < 0 || c >= A.n || (p > b && A.ci[p - 1] >= c)) f |= 2;
            if (!isfinite(A.v[p])) f |= 4;
        }
    }
    if (i == A.n - 1 && e != nnz) f |= 1;
    if (f) atomicOr(flag, f);
}

hipError_t validate_csr(CsrView A, int64_t nnz, int *flag, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    int wpb = 4;
    hipLaunchKernelGGL(k_validate, dim3((A.n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, A, nnz,
                       flag);
    return hipGetLastError();
}

constexpr int kRedBlock = 256;

// Fixed-order block reduction (wave butterflies, then the wave sums in order).
__device__ double block_sum(double s) {
    __shared__ double ws[kRedBlock / kWave];
    s = wave_sum(s);
    if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int j = 0; j < kRedBlock / kWave; j++) t += ws[j];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kRedBlock) void k_sumsq_part(const double *v, const int64_t *count,
                                                          int64_t maxcount, double *part) {
    int64_t m = count ? *count : maxcount;
    double s = 0;
    int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t j = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; j < m; j += stride) {
        double x = v[j];
        s = fma(x, x, s);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedBlock) void k_sum_parts(const double *part, int nparts,
                                                         double *out) {
    double s = 0;
    for (int j = threadIdx.x; j < nparts; j += kRedBlock) s += part[j];
    s = block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// Partial-sum blocks for m values: about 16 values per thread, at most
// nparts; a function of the size alone, so sums are reproducible.
static int parts_for(int64_t m, int nparts) {
    const int64_t want = (m + (int64_t)kRedBlock * 16 - 1) / ((int64_t)kRedBlock * 16);
    return (int)(want < 1 ? 1 : want < nparts ? want : nparts);
}

hipError_t sumsq(const double *v, const int64_t *count, int64_t maxcount, double *part, int nparts,
                 double *out, hipStream_t st) {
    nparts = parts_for(maxcount, nparts);
    hipLaunchKernelGGL(k_sumsq_part, dim3(nparts), dim3(kRedBlock), 0, st, v, count, maxcount,
                       part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kRedBlock), 0, st, part, nparts, out);
    return hipGetLastError();
}

__global__ void k_scale_ldexp(const double *in, double *out, int64_t m, int e) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) out[j] = ldexp(in[j], e);
}

hipError_t scale_ldexp(const double *in, double *out, int64_t m, int e, hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_ldexp, dim3((m + 255) / 256), dim3(256), 0, st, in, out, m, e);
    return hipGetLastError();
}

__global__ void k_negate(double *v, int64_t m) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) v[j] = -v[j];
}

hipError_t negate_values(double *v, int64_t m, hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_negate, dim3((m + 255) / 256), dim3(256), 0, st, v, m);
    return hipGetLastError();
}

__global__ __launch_bounds__(kRedBlock) void k_sum_part(const double *v, int64_t m,
                                                        double *part) {
    double s = 0;
    int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t j = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; j < m; j += stride) s += v[j];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t sum_values(const double *v, int64_t m, double *part, int nparts, double *out,
                      hipStream_t st) {
    nparts = parts_for(m, nparts);
    hipLaunchKernelGGL(k_sum_part, dim3(nparts), dim3(kRedBlock), 0, st, v, m, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kRedBlock), 0, st, part, nparts, out);
    return hipGetLastError();
}

__global__ void k_add_ldexp(const double *a, const double *b, double *out, int64_t m, int e) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) out[j] = ldexp(a[j] + b[j], e);
}

hipError_t add_scaled_ldexp(const double *a, const double *b, double *out, int64_t m, int e,
                            hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_ldexp, dim3((m + 255) / 256), dim3(256), 0, st, a, b, out, m, e);
    return hipGetLastError();
}

__global__ void k_compare(CsrView A, CsrView B, int64_t nnz, int *flags) {
    // Grid-stride; each wave clears a flag with one atomic, and only when
    // one of its lanes found a mismatch.
    bool pat = false, eq = true, neg = true;
    const int64_t m = nnz > A.n + 1 ? nnz : A.n + 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
        if (j <= A.n && A.rp[j] != B.rp[j]) pat = true;
        if (j < nnz) {
            if (A.ci[j] != B.ci[j]) pat = true;
            const double a = A.v[j], b = B.v[j];
            if (a != b) eq = false;
            if (a != -b) neg = false;
        }
    }
    const unsigned long long bp = __ballot(pat), be = __ballot(!eq), bn = __ballot(!neg);
    if (lane_id() == 0) {
        if (bp) atomicAnd(&flags[0], 0);
        if (be) atomicAnd(&flags[1], 0);
        if (bn) atomicAnd(&flags[2], 0);
    }
}

hipError_t compare_csr(CsrView A, CsrView B, int64_t nnz, int *flags, hipStream_t st) {
    int64_t m = nnz > A.n + 1 ? nnz : A.n + 1;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_compare, dim3((unsigned)blocks), dim3(256), 0, st, A, B, nnz, flags);
    return hipGetLastError();
}

// ============================================================== filter (Algorithm 4.1)

__global__ void k_filter_init(FilterCtl *c, double eg_scale, const double *norm2, double er,
                              int maxit) {
    double eg = norm2 ? eg_scale * sqrt(*norm2) : eg_scale;
    c->eg = eg;
    c->er = er;
    c->maxit = maxit;
    c->iter = 0;
    c->status = 0;
    c->b = INFINITY;
    c->m = 1.0;                       // m_0 = 1
    c->arrive = 0;
    if (eg > 0.0) {
        c->theta = eg;                // eps_f^(1) = eps_g / m_0
        c->done = 0;
    } else {
        c->theta = 0.0;               // a = 0: only exact zeros leave
        c->b = 0.0;
        c->done = 1;
    }
}

__global__ void k_filter_theta(FilterCtl *c, double theta) {
    c->eg = 0.0;
    c->theta = theta;
    c->iter = 0;
    c->status = 0;
    c->done = 1;
    c->arrive = 0;
}

hipError_t filter_init(FilterCtl *c, double eg_scale, const double *norm2, double er, int maxit,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_filter_init, dim3(1), dim3(1), 0, st, c, eg_scale, norm2, er, maxit);
    return hipGetLastError();
}

hipError_t filter_init_theta(FilterCtl *c, double theta, hipStream_t st) {
    hipLaunchKernelGGL(k_filter_theta, dim3(1), dim3(1), 0, st, c, theta);
    return hipGetLastError();
}

// End of one pass: this block's partial s goes to part[]; the last block to
// finish sums the block partials in a fixed order and advances the
// controller: m = b / theta and the next theta = eps_g / m, or stop when
// b <= eps_g (1 + e_r).
__device__ void filter_pass_end(double s, double theta, FilterCtl *c, double *part);

// One pass: b^2 = sum of v^2 over |v| <= theta (the entries still in the
// drop vector b_n of Algorithm 4.1, since theta only decreases).
__global__ __launch_bounds__(kRedBlock) void k_filter_pass(const double *__restrict__ v,
                                                           const int64_t *count,
                                                           int64_t maxcount, FilterCtl *c,
                                                           double *part) {
    if (c->done) return;
    const double theta = c->theta;
    const int64_t m = count ? *count : maxcount;
    double s = 0.0;
    int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t j = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; j < m; j += stride) {
        double x = v[j];
        if (fabs(x) <= theta) s = fma(x, x, s);
    }
    filter_pass_end(s, theta, c, part);
}

// The pass over candidate tiles: one wave per tile (grid-stride), each lane
// 32 contiguous bytes.
__global__ __launch_bounds__(kRedBlock) void k_filter_pass_tiles(const double *__restrict__ tiles,
                                                                 const double *__restrict__ tmin,
                                                                 const double *__restrict__ tmax,
                                                                 const double *__restrict__ tsq,
                                                                 int64_t ntiles, FilterCtl *c,
                                                                 double *part,
                                                                 uint4 *__restrict__ krc,
                                                                 const int64_t *__restrict__ tmir) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    if (c->done) return;
    const double theta = c->theta;
    constexpr int wpb = kRedBlock / kWave;
    const int lane = lane_id();
    double s = 0.0;
    // the tile entries at or below theta and their counts above it, per row;
    // a tile with a mirror (tmir >= 0: the candidate is symmetric, the
    // mirror its transpose) counts twice, and the mirror's row counts are
    // this tile's column counts
    auto take = [&](const v4 &x, int64_t t, int64_t mir) {
        uint32_t w[4];
        const double wt = mir >= 0 ? 2.0 : 1.0;
        int cc = 0;   // entries above theta in column lane % 16 of this lane's rows
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (fabs(x[r]) <= theta) s = fma(wt * x[r], x[r], s);
            cc += fabs(x[r]) > theta;
            // entries above theta per tile row: lane l holds row l / 16 + 4 r
            // (column l % 16), so each 16-lane group of the ballot is one row
            const unsigned long long k = __ballot(fabs(x[r]) > theta);
            w[r] = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g)
                w[r] |= (uint32_t)__popcll((k >> (16 * g)) & 0xffffull) << (8 * g);
        }
        if (krc && lane == 0) krc[t] = make_uint4(w[0], w[1], w[2], w[3]);
        if (krc && mir >= 0) {
            cc += __shfl_xor(cc, 16);
            cc += __shfl_xor(cc, 32);   // lane l: column l % 16's count
            uint32_t u[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int col = 0; col < 16; ++col)
                u[col >> 2] |= (uint32_t)__builtin_amdgcn_readlane(cc, col) << (8 * (col & 3));
            if (lane == 0) krc[mir] = make_uint4(u[0], u[1], u[2], u[3]);
        }
    };
    // each wave takes 64 consecutive tiles at a time: one lane per tile
    // reads its summaries (a tile wholly at or below theta adds its stored
    // sum of squares), then the tiles in between are read in order with the
    // next one's load in flight
    // (with tmir, the tiles marked -2, mirrors of others, are left out)
    const int64_t nchunk = (ntiles + kWave - 1) / kWave;
    for (int64_t q = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; q < nchunk;
         q += (int64_t)gridDim.x * wpb) {
        const int64_t t0 = q * kWave, t = t0 + lane;
        bool mid = false;
        int64_t mir = -1;
        if (t < ntiles) mir = tmir ? tmir[t] : -1;
        if (t < ntiles && mir != -2 && tmin[t] <= theta) {   // something at or below theta
            if (tmax[t] <= theta)
                s += (mir >= 0 ? 2.0 : 1.0) * tsq[t];      // everything at or below theta
            else
                mid = true;
        }
        unsigned long long m = __ballot(mid);
        if (!m) continue;
        int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        int64_t tt = t0 + l;
        v4 x = *(const v4 *)(tiles + tt * 256 + 4 * lane);
        for (;;) {
            const bool more = m != 0;
            int64_t tt2 = tt;
            v4 x2 = x;
            if (more) {
                l = __ffsll((long long)m) - 1;
                m &= m - 1;
                tt2 = t0 + l;
                x2 = *(const v4 *)(tiles + tt2 * 256 + 4 * lane);
            }
            const int64_t mt = tmir ? tmir[tt] : -1;
            take(x, tt, mt);
            if (!more) break;
            tt = tt2;
            x = x2;
        }
    }
    filter_pass_end(s, theta, c, part);
}

__device__ void filter_pass_end(double s, double theta, FilterCtl *c, double *part) {
    s = block_sum(s);
    __shared__ unsigned ticket;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        __threadfence();
        ticket = atomicAdd(&c->arrive, 1u);
    }
    __syncthreads();
    if (ticket != gridDim.x - 1) return;
    __threadfence();
    double t = 0.0;
    for (int j = threadIdx.x; j < (int)gridDim.x; j += kRedBlock)
        t += __builtin_nontemporal_load(&part[j]);
    t = block_sum(t);
    if (threadIdx.x == 0) {
        double b = sqrt(t);
        c->b = b;
        c->iter += 1;
        c->arrive = 0;
        if (b <= c->eg * (1.0 + c->er)) {
            c->done = 1;
        } else if (c->iter >= c->maxit) {
            c->done = 1;
            c->status = 1;
        } else {
            c->m = b / theta;
            c->theta = c->eg / c->m;
        }
    }
}

hipError_t filter_pass_tiles(const double *tiles, const double *tmin, const double *tmax,
                             const double *tsq, int64_t ntiles, FilterCtl *c, double *part,
                             int nparts, uint4 *krc, hipStream_t st, const int64_t *tmir) {
    nparts = parts_for(ntiles * 16, nparts);
    hipLaunchKernelGGL(k_filter_pass_tiles, dim3(nparts), dim3(kRedBlock), 0, st, tiles, tmin,
                       tmax, tsq, ntiles, c, part, krc, tmir);
    return hipGetLastError();
}

hipError_t filter_pass(const double *v, const int64_t *count, int64_t maxcount, FilterCtl *c,
                       double *part, int nparts, hipStream_t st) {
    nparts = parts_for(maxcount, nparts);
    hipLaunchKernelGGL(k_filter_pass, dim3(nparts), dim3(kRedBlock), 0, st, v, count, maxcount, c,
                       part);
    return hipGetLastError();
}

// ============================================================== compaction

__device__ __forceinline__ unsigned long long lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Per row: entries kept (|v| > theta); with addI the diagonal becomes 1 + v
// (dropped if exactly 0) or is inserted as 1.
__global__ void k_count_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                             const FilterCtl *c, int addI, int64_t *cnt,
                             const int32_t *row_inst, const int *inst_addI) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    if (row_inst) {
        const int k = row_inst[i];
        c += k;
        addI = inst_addI ? inst_addI[k] : addI;
    }
    const double theta = c->theta;
    long long k = 0;
    int dstate = 0;   // 0 absent/dropped, 1 kept, 2 kept but 1 + v == 0
    for (int64_t p = crp[i] + lane_id(); p < crp[i + 1]; p += kWave) {
        double x = cv[p];
        bool keep = fabs(x) > theta;
        k += keep;
        if (addI && cci[p] == i && keep) dstate = (x + 1.0 == 0.0) ? 2 : 1;
    }
    k = wave_sum_ll(k);
    if (addI) dstate = wave_max(dstate);
    if (lane_id() == 0) cnt[i] = k + (addI ? (dstate == 0 ? 1 : (dstate == 2 ? -1 : 0)) : 0);
}

__global__ void k_write_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                             const FilterCtl *c, int addI, const int64_t *orp, int32_t *oci,
                             double *ov, const int32_t *row_inst, const int *inst_addI) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    if (row_inst) {
        const int k = row_inst[i];
        c += k;
        addI = inst_addI ? inst_addI[k] : addI;
    }
    const double theta = c->theta;
    const int64_t b = crp[i], e = crp[i + 1];
    // diagonal state (see k_count_kept)
    int dstate = 0;
    if (addI) {
        for (int64_t p = b + lane_id(); p < e; p += kWave) {
            double x = cv[p];
            if (cci[p] == i && fabs(x) > theta) dstate = (x + 1.0 == 0.0) ? 2 : 1;
        }
        dstate = wave_max(dstate);
    }
    const bool insert = addI && dstate == 0;
    int64_t out = orp[i];
    int64_t written = 0;
    bool inserted = false;
    for (int64_t p0 = b; p0 < e; p0 += kWave) {
        int64_t p = p0 + lane_id();
        bool valid = p < e;
        int col = valid ? cci[p] : 0;
        double x = valid ? cv[p] : 0.0;
        bool keep = valid && fabs(x) > theta;
        if (addI && keep && col == i) {
            x += 1.0;
            if (x == 0.0) keep = false;
        }
        if (insert && !inserted) {
            // the identity entry goes before the first column > i
            unsigned long long after = __ballot(valid && col > i);
            unsigned long long pre = __ballot(keep && col < i);
            if (after) {
                int64_t pos = written + __popcll(pre);
                if (lane_id() == 0) {
                    oci[out + pos] = (int32_t)i;
                    ov[out + pos] = 1.0;
                }
                inserted = true;
                unsigned long long km = __ballot(keep);
                int64_t my = written + __popcll(km & lanemask_lt()) + (col > i ? 1 : 0);
                if (keep) {
                    oci[out + my] = col;
                    ov[out + my] = x;
                }
                written += __popcll(km) + 1;
                continue;
            }
        }
        unsigned long long km = __ballot(keep);
        int64_t my = written + __popcll(km & lanemask_lt());
        if (keep) {
            oci[out + my] = col;
            ov[out + my] = x;
        }
        written += __popcll(km);
    }
    if (insert && !inserted && lane_id() == 0) {
        oci[out + written] = (int32_t)i;
        ov[out + written] = 1.0;
    }
}

hipError_t count_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                      const FilterCtl *c, int addI, int64_t *cnt, hipStream_t st,
                      const int32_t *row_inst, const int *inst_addI) {
    if (n == 0) return hipSuccess;
    int wpb = 4;
    hipLaunchKernelGGL(k_count_kept, dim3((n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, crp,
                       cci, cv, n, c, addI, cnt, row_inst, inst_addI);
    return hipGetLastError();
}

hipError_t write_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                      const FilterCtl *c, int addI, const int64_t *orp, int32_t *oci, double *ov,
                      hipStream_t st, const int32_t *row_inst, const int *inst_addI) {
    if (n == 0) return hipSuccess;
    int wpb = 4;
    hipLaunchKernelGGL(k_write_kept, dim3((n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, crp,
                       cci, cv, n, c, addI, orp, oci, ov, row_inst, inst_addI);
    return hipGetLastError();
}

// ============================================================== sparse add
// One thread per row merges the two sorted rows.

__global__ void k_add(CsrView A, CsrView B, int64_t *cnt, const int64_t *crp, int32_t *cci,
                      double *cv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int64_t p = A.rp[i], pe = A.rp[i + 1], q = B.rp[i], qe = B.rp[i + 1];
    int64_t o = crp ? crp[i] : 0, k = 0;
    while (p < pe || q < qe) {
        int ja = p < pe ? A.ci[p] : INT32_MAX;
        int jb = q < qe ? B.ci[q] : INT32_MAX;
        int j;
        double s;
        if (ja == jb) {
            j = ja;
            s = A.v[p++] + B.v[q++];
        } else if (ja < jb) {
            j = ja;
            s = A.v[p++];
        } else {
            j = jb;
            s = B.v[q++];
        }
        if (s == 0.0) continue;
        if (crp) {
            cci[o + k] = j;
            cv[o + k] = s;
        }
        k++;
    }
    if (!crp) cnt[i] = k;
}

hipError_t add_count(CsrView A, CsrView B, int64_t *cnt, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((A.n + 127) / 128), dim3(128), 0, st, A, B, cnt,
                       (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr);
    return hipGetLastError();
}

hipError_t add_write(CsrView A, CsrView B, const int64_t *crp, int32_t *cci, double *cv,
                     hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((A.n + 127) / 128), dim3(128), 0, st, A, B, (int64_t *)nullptr,
                       crp, cci, cv);
    return hipGetLastError();
}

// One wave per row.  The distinct columns of the row over all terms are
// marked in a bit map over the row's column window (prefix counts give each
// its rank); the terms then add into an accumulator per rank, one term after
// the other, and the nonzero sums are counted or written in column order.
constexpr int kSumBatch = 8;      // terms whose first chunks load together
constexpr int kSumWaves = 4;      // rows per workgroup
constexpr int kSumWords = 512;    // bit-map words per wave (16384 columns)
constexpr int kSumAcc = 256;      // distinct columns per wave (sparse rows)
constexpr int kSumDense = 1024;   // column block of a dense row (8 KB of LDS)
static_assert(kSumWords * 8 + kSumAcc * 12 <= kSumDense * 8, "sparse row slice fits");

__device__ __forceinline__ int64_t readlane_i64_(int64_t x, int j) {
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffff), j);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), j);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Per row: the global scratch bytes a row needs when its column window
// exceeds the LDS bit map, else 0.
__global__ void k_sum_bounds(SumTerms T, int64_t n, int64_t *bytes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int mn = INT32_MAX, mx = -1;
    int64_t ub = 0;
    for (int t = 0; t < T.m; ++t) {
        const int64_t b = T.rp[t][i], e = T.rp[t][i + 1];
        if (e > b) {
            mn = min(mn, T.ci[t][b]);
            mx = max(mx, T.ci[t][e - 1]);
            ub += e - b;
        }
    }
    int64_t need = 0;
    if (mx >= 0) {
        const int64_t W = ((mx - (mn & ~31)) >> 5) + 1;
        if (W > kSumWords) need = (8 * W + 12 * ub + 255) & ~int64_t(255);
    }
    bytes[i] = need;
}

template <bool kWrite>
__global__ __launch_bounds__(kWave * kSumWaves) void k_sum_terms(SumTerms T, int64_t n,
                                                                  int64_t *cnt, int *overflow,
                                                                  const int64_t *orp,
                                                                  int32_t *oci, double *ov,
                                                                  char *gscr,
                                                                  const int64_t *goff) {
    // one LDS slice per wave: the bit map, accumulator and columns of a
    // sparse row, or the dense accumulator of a column block
    __shared__ double slds[kSumWaves][kSumDense];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * kSumWaves + wv;
    if (i >= n) return;
    // rows too wide for the LDS bit map work in their own global scratch
    const bool big = goff[i + 1] > goff[i];
    auto sync_wave = [big]() {
        if (big) __threadfence();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    };
    int mn = INT32_MAX, mx = -1;
    int64_t ub = 0;
    int64_t tb = 0, te = 0;   // lane t < m: term t's entries of row i
    if (lane < T.m) {
        tb = T.rp[lane][i];
        te = T.rp[lane][i + 1];
        if (te > tb) {
            mn = T.ci[lane][tb];
            mx = T.ci[lane][te - 1];
            ub = te - tb;
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    ub = wave_sum_ll(ub);
    if (mx < 0) {
        if (!kWrite && lane == 0) cnt[i] = 0;
        return;
    }
    const int lo = mn & ~31;
    const int W = ((mx - lo) >> 5) + 1;
    if (!big && W > kSumWords) {   // the bounds disagree: not summed
        if (!kWrite && lane == 0) {
            cnt[i] = 0;
            atomicOr(overflow, 1);
        }
        return;
    }
    if (!big && ub > kSumAcc) {
        // Many distinct columns in a narrow window: dense accumulation in
        // blocks of kSumDense columns, each starting at the smallest column
        // not yet taken (lane t < m keeps term t's position).
        double *acc = slds[wv];
        const int tl = lane < T.m ? lane : 0;   // in-range term index
        int64_t cur = lane < T.m ? T.rp[tl][i] : 0;
        const int64_t end = lane < T.m ? T.rp[tl][i + 1] : 0;
        long long kept = 0;
        int64_t o = kWrite ? orp[i] : 0;
        for (;;) {
            const int head = cur < end ? T.ci[tl][cur] : INT32_MAX;
            const int c0 = wave_min(head);
            if (c0 == INT32_MAX) break;
            for (int r = lane; r < kSumDense; r += kWave) acc[r] = 0.0;
            sync_wave();
            for (int t = 0; t < T.m; ++t) {
                int64_t b = readlane_i64_(cur, t);
                const int64_t e = readlane_i64_(end, t);
                for (;;) {
                    const int64_t p = b + lane;
                    const int c = p < e ? T.ci[t][p] : INT32_MAX;
                    const bool in = (int64_t)c < (int64_t)c0 + kSumDense;
                    if (in) acc[c - c0] += T.v[t][p];
                    const int k = __popcll(__ballot(in));
                    b += k;
                    if (k < kWave) break;
                }
                if (lane == t) cur = b;
                sync_wave();
            }
            for (int r0 = 0; r0 < kSumDense; r0 += kWave) {
                const int r = r0 + lane;
                const bool keep = acc[r] != 0.0;
                const unsigned long long bm = __ballot(keep);
                if (kWrite && keep) {
                    const int64_t q = o + __popcll(bm & ((1ull << lane) - 1ull));
                    oci[q] = c0 + r;
                    ov[q] = acc[r];
                }
                o += __popcll(bm);
                kept += __popcll(bm);
            }
            sync_wave();
        }
        if (!kWrite && lane == 0) cnt[i] = kept;
        return;
    }
    uint2 *bits = big ? (uint2 *)(gscr + goff[i]) : (uint2 *)slds[wv];
    double *acc = big ? (double *)(bits + W) : (double *)(bits + kSumWords);
    int32_t *col = big ? (int32_t *)(acc + ub) : (int32_t *)(acc + kSumAcc);
    for (int w = lane; w < W; w += kWave) bits[w] = make_uint2(0u, 0u);
    sync_wave();
    // the first 64 entries of kSumBatch terms are loaded together; longer
    // term rows continue one chunk at a time
    for (int t0 = 0; t0 < T.m; t0 += kSumBatch) {
        int c[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int t = t0 + u;
            c[u] = -1;
            if (t < T.m) {
                const int64_t p = readlane_i64_(tb, t) + lane;
                if (p < readlane_i64_(te, t)) c[u] = T.ci[t][p];
            }
        }
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            if (c[u] >= 0) {
                const int d = c[u] - lo;
                atomicOr(&bits[d >> 5].x, 1u << (d & 31));
            }
            const int t = t0 + u;
            if (t >= T.m) continue;
            const int64_t e = readlane_i64_(te, t);
            for (int64_t p = readlane_i64_(tb, t) + kWave + lane; p < e; p += kWave) {
                const int d = T.ci[t][p] - lo;
                atomicOr(&bits[d >> 5].x, 1u << (d & 31));
            }
        }
    }
    sync_wave();
    unsigned carry = 0;
    for (int w0 = 0; w0 < W; w0 += kWave) {
        const int w = w0 + lane;
        const unsigned pc = w < W ? __popc(bits[w].x) : 0u;
        const unsigned inc = wave_incl_scan(pc);
        if (w < W) bits[w].y = carry + inc - pc;
        carry += __shfl(inc, kWave - 1);
    }
    const int U = (int)carry;
    for (int r = lane; r < U; r += kWave) acc[r] = 0.0;
    sync_wave();
    auto rank = [&](int c) {
        const int d = c - lo;
        const uint2 e2 = bits[d >> 5];
        return (int)(e2.y + __popc(e2.x & ((1u << (d & 31)) - 1u)));
    };
    // terms in order; within one term a row's columns are distinct.  The
    // first 64 entries of kSumBatch terms are loaded together.
    for (int t0 = 0; t0 < T.m; t0 += kSumBatch) {
        int c[kSumBatch];
        double v[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int t = t0 + u;
            c[u] = -1;
            v[u] = 0.0;
            if (t < T.m) {
                const int64_t p = readlane_i64_(tb, t) + lane;
                if (p < readlane_i64_(te, t)) {
                    c[u] = T.ci[t][p];
                    v[u] = T.v[t][p];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int t = t0 + u;
            if (t >= T.m) break;
            if (c[u] >= 0) {
                const int r = rank(c[u]);
                acc[r] += v[u];
                col[r] = c[u];
            }
            const int64_t e = readlane_i64_(te, t);
            for (int64_t p = readlane_i64_(tb, t) + kWave + lane; p < e; p += kWave) {
                const int cc = T.ci[t][p];
                const int r = rank(cc);
                acc[r] += T.v[t][p];
                col[r] = cc;
            }
            sync_wave();
        }
    }
    if (!kWrite) {
        long long k = 0;
        for (int r = lane; r < U; r += kWave) k += acc[r] != 0.0;
        k = wave_sum_ll(k);
        if (lane == 0) cnt[i] = k;
        return;
    }
    int64_t o = orp[i];
    for (int r0 = 0; r0 < U; r0 += kWave) {
        const int r = r0 + lane;
        const bool keep = r < U && acc[r] != 0.0;
        const unsigned long long bm = __ballot(keep);
        if (keep) {
            const int64_t q = o + __popcll(bm & ((1ull << lane) - 1ull));
            oci[q] = col[r];
            ov[q] = acc[r];
        }
        o += __popcll(bm);
    }
}

hipError_t sum_terms_bounds(const SumTerms &T, int64_t n, int64_t *bytes, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_bounds, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, T, n,
                       bytes);
    return hipGetLastError();
}

hipError_t sum_terms_count(const SumTerms &T, int64_t n, char *gscr, const int64_t *goff,
                           int64_t *cnt, int *overflow, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_terms<false>, dim3((unsigned)((n + kSumWaves - 1) / kSumWaves)),
                       dim3(kWave * kSumWaves), 0, st, T, n, cnt, overflow,
                       (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr, gscr,
                       goff);
    return hipGetLastError();
}

hipError_t sum_terms_write(const SumTerms &T, int64_t n, char *gscr, const int64_t *goff,
                           const int64_t *orp, int32_t *oci, double *ov, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_terms<true>, dim3((unsigned)((n + kSumWaves - 1) / kSumWaves)),
                       dim3(kWave * kSumWaves), 0, st, T, n, (int64_t *)nullptr, (int *)nullptr,
                       orp, oci, ov, gscr, goff);
    return hipGetLastError();
}

// Values of E = I + T (exact zeros dropped) at T's entries.  Row by row the
// two patterns differ at most at the diagonal: E has one entry more when T
// has no diagonal entry, one fewer when T's diagonal entry was -1.
__global__ void k_values_at_t(const int64_t *trp, const int32_t *tci, const int64_t *erp,
                              const double *ev, int64_t n, double *out) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const int64_t tb = trp[i], te = trp[i + 1], eb = erp[i];
    const int64_t delta = (erp[i + 1] - eb) - (te - tb);   // +1, 0 or -1
    for (int64_t q = tb + lane_id(); q < te; q += kWave) {
        const int c = tci[q];
        int64_t pos = q - tb;
        if (delta != 0 && c > i) pos += delta;
        out[q] = delta < 0 && c == i ? 0.0 : ev[eb + pos];
    }
}

hipError_t values_at_t(const int64_t *trp, const int32_t *tci, const int64_t *erp,
                       const double *ev, int64_t n, double *out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_values_at_t, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, trp, tci,
                       erp, ev, n, out);
    return hipGetLastError();
}

__global__ void k_identity(int64_t n, int64_t *rp, int32_t *ci, double *v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rp[i] = i;
    if (i < n) {
        ci[i] = (int32_t)i;
        v[i] = 1.0;
    }
}

hipError_t fill_identity(int64_t n, int64_t *rp, int32_t *ci, double *v, hipStream_t st) {
    hipLaunchKernelGGL(k_identity, dim3((n + 256) / 256), dim3(256), 0, st, n, rp, ci, v);
    return hipGetLastError();
}

// ============================================================== transpose
// Counting sort by column with atomic slot assignment, then every row of the
// transpose is sorted by its column index so the result is canonical.

__global__ void k_colcount(CsrView A, int64_t nnz, int64_t *colcnt) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= A.n) return;
    for (int64_t p = A.rp[i] + lane_id(); p < A.rp[i + 1]; p += kWave)
        atomicAdd((unsigned long long *)&colcnt[A.ci[p]], 1ull);
}

// The payload of each transposed entry: its value (V = double) or its
// position in A (V = int64_t).
template <typename V>
__global__ void k_colfill(CsrView A, int64_t *fillpos, int32_t *tci, V *tv) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= A.n) return;
    for (int64_t p = A.rp[i] + lane_id(); p < A.rp[i + 1]; p += kWave) {
        int64_t d = (int64_t)atomicAdd((unsigned long long *)&fillpos[A.ci[p]], 1ull);
        tci[d] = (int32_t)i;
        if constexpr (std::is_same<V, double>::value)
            tv[d] = A.v[p];
        else
            tv[d] = p;
    }
}

// One wave per row: each entry of the unsorted row (uci, uv) goes to its rank
// among the row's columns (distinct within a row) in (ci, v).  Keys of rows
// up to kRankLds entries are staged in LDS; longer rows are ranked from
// memory.
constexpr int kRankLds = 1024;

template <typename V>
__global__ __launch_bounds__(256) void k_rank_rows(const int64_t *rp, int64_t n,
                                                   const int32_t *uci, const V *uv,
                                                   int32_t *ci, V *v) {
    __shared__ int32_t skey[4][kRankLds];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + wv;
    if (i >= n) return;
    const int64_t b = rp[i], len = rp[i + 1] - b;
    if (len <= kRankLds) {
        int32_t *k = skey[wv];
        for (int64_t t = lane; t < len; t += kWave) k[t] = uci[b + t];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int64_t t = lane; t < len; t += kWave) {
            const int32_t x = k[t];
            int64_t r = 0;
            for (int64_t u = 0; u < len; ++u) r += k[u] < x;
            ci[b + r] = x;
            v[b + r] = uv[b + t];
        }
    } else {
        for (int64_t t = lane; t < len; t += kWave) {
            const int32_t x = uci[b + t];
            int64_t r = 0;
            for (int64_t u = 0; u < len; ++u) r += uci[b + u] < x;
            ci[b + r] = x;
            v[b + r] = uv[b + t];
        }
    }
}

template <typename V>
static hipError_t transpose_t(CsrView A, int64_t nnz, int64_t *trp, int32_t *tci, V *tv,
                              int64_t *colcnt, int64_t *fillpos, int32_t *tmp_ci, V *tmp_v,
                              void *scan_tmp, size_t scan_tmp_bytes_, hipStream_t st) {
    int64_t n = A.n;
    hipError_t e = hipMemsetAsync(colcnt, 0, sizeof(int64_t) * (n > 0 ? n : 1), st);
    if (e != hipSuccess || n == 0) {
        if (n == 0) return hipMemsetAsync(trp, 0, sizeof(int64_t), st);
        return e;
    }
    int wpb = 4;
    dim3 g((n + wpb - 1) / wpb), b(wpb * kWave);
    hipLaunchKernelGGL(k_colcount, g, b, 0, st, A, nnz, colcnt);
    e = scan_i64(colcnt, trp, n, scan_tmp, scan_tmp_bytes_, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(fillpos, trp, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    // unsorted rows into the scratch arrays, then each entry to its rank
    hipLaunchKernelGGL(k_colfill<V>, g, b, 0, st, A, fillpos, tmp_ci, tmp_v);
    hipLaunchKernelGGL(k_rank_rows<V>, dim3((n + 3) / 4), dim3(256), 0, st, trp, n, tmp_ci,
                       tmp_v, tci, tv);
    return hipGetLastError();
}

hipError_t transpose(CsrView A, int64_t nnz, int64_t *trp, int32_t *tci, double *tv,
                     int64_t *colcnt, int64_t *fillpos, int32_t *tmp_ci, double *tmp_v,
                     void *scan_tmp, size_t scan_tmp_bytes_, hipStream_t st) {
    return transpose_t<double>(A, nnz, trp, tci, tv, colcnt, fillpos, tmp_ci, tmp_v, scan_tmp,
                               scan_tmp_bytes_, st);
}

hipError_t transpose_index(CsrView A, int64_t nnz, int64_t *trp, int32_t *tci, int64_t *tpos,
                           int64_t *colcnt, int64_t *fillpos, int32_t *tmp_ci, int64_t *tmp_pos,
                           void *scan_tmp, size_t scan_tmp_bytes_, hipStream_t st) {
    return transpose_t<int64_t>(A, nnz, trp, tci, tpos, colcnt, fillpos, tmp_ci, tmp_pos,
                                scan_tmp, scan_tmp_bytes_, st);
}

}  // namespace xpm

namespace xpm {

// ============================================================== complex values
// A complex entry is a double2 (real, imaginary).  Its modulus is
// sqrt(re^2 + im^2) with each product and the sum rounded once (no fused
// multiply-add), and Algorithm 4.1 sums the squared moduli of the dropped
// entries.

__device__ __forceinline__ double mod2_z(double2 z) {
#pragma clang fp contract(off)
    return z.x * z.x + z.y * z.y;
}

__global__ __launch_bounds__(kRedBlock) void k_filter_pass_z(const double2 *__restrict__ v,
                                                             const int64_t *count,
                                                             int64_t maxcount, FilterCtl *c,
                                                             double *part) {
    if (c->done) return;
    const double theta = c->theta;
    const int64_t m = count ? *count : maxcount;
    double s = 0.0;
    int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t j = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; j < m; j += stride) {
        const double q = mod2_z(v[j]);
        if (sqrt(q) <= theta) s += q;
    }
    filter_pass_end(s, theta, c, part);
}

hipError_t filter_pass_z(const double *v, const int64_t *count, int64_t maxcount, FilterCtl *c,
                         double *part, int nparts, hipStream_t st) {
    nparts = parts_for(maxcount, nparts);
    hipLaunchKernelGGL(k_filter_pass_z, dim3(nparts), dim3(kRedBlock), 0, st, (const double2 *)v,
                       count, maxcount, c, part);
    return hipGetLastError();
}

// Kept entries (|z| > theta) per row; with addI the diagonal becomes 1 + z
// (dropped if exactly 0) or is inserted as 1.
__global__ void k_count_kept_z(const int64_t *crp, const int32_t *cci, const double2 *cv,
                               int64_t n, const FilterCtl *c, int addI, int64_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const double theta = c->theta;
    long long k = 0;
    int dstate = 0;   // 0 absent/dropped, 1 kept, 2 kept but 1 + z == 0
    for (int64_t p = crp[i] + lane_id(); p < crp[i + 1]; p += kWave) {
        const double2 x = cv[p];
        const bool keep = sqrt(mod2_z(x)) > theta;
        k += keep;
        if (addI && cci[p] == i && keep) dstate = (x.x + 1.0 == 0.0 && x.y == 0.0) ? 2 : 1;
    }
    k = wave_sum_ll(k);
    if (addI) dstate = wave_max(dstate);
    if (lane_id() == 0) cnt[i] = k + (addI ? (dstate == 0 ? 1 : (dstate == 2 ? -1 : 0)) : 0);
}

__global__ void k_write_kept_z(const int64_t *crp, const int32_t *cci, const double2 *cv,
                               int64_t n, const FilterCtl *c, int addI, const int64_t *orp,
                               int32_t *oci, double2 *ov) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const double theta = c->theta;
    const int64_t b = crp[i], e = crp[i + 1];
    int dstate = 0;
    if (addI) {
        for (int64_t p = b + lane_id(); p < e; p += kWave) {
            const double2 x = cv[p];
            if (cci[p] == i && sqrt(mod2_z(x)) > theta)
                dstate = (x.x + 1.0 == 0.0 && x.y == 0.0) ? 2 : 1;
        }
        dstate = wave_max(dstate);
    }
    const bool insert = addI && dstate == 0;
    const int64_t out = orp[i];
    int64_t written = 0;
    bool inserted = false;
    for (int64_t p0 = b; p0 < e; p0 += kWave) {
        const int64_t p = p0 + lane_id();
        const bool valid = p < e;
        const int col = valid ? cci[p] : 0;
        double2 x = valid ? cv[p] : make_double2(0.0, 0.0);
        bool keep = valid && sqrt(mod2_z(x)) > theta;
        if (addI && keep && col == i) {
            x.x += 1.0;
            if (x.x == 0.0 && x.y == 0.0) keep = false;
        }
        if (insert && !inserted) {
            // the identity entry goes before the first column > i
            const unsigned long long after = __ballot(valid && col > i);
            const unsigned long long pre = __ballot(keep && col < i);
            if (after) {
                const int64_t pos = written + __popcll(pre);
                if (lane_id() == 0) {
                    oci[out + pos] = (int32_t)i;
                    ov[out + pos] = make_double2(1.0, 0.0);
                }
                inserted = true;
                const unsigned long long km = __ballot(keep);
                const int64_t my = written + __popcll(km & lanemask_lt()) + (col > i ? 1 : 0);
                if (keep) {
                    oci[out + my] = col;
                    ov[out + my] = x;
                }
                written += __popcll(km) + 1;
                continue;
            }
        }
        const unsigned long long km = __ballot(keep);
        const int64_t my = written + __popcll(km & lanemask_lt());
        if (keep) {
            oci[out + my] = col;
            ov[out + my] = x;
        }
        written += __popcll(km);
    }
    if (insert && !inserted && lane_id() == 0) {
        oci[out + written] = (int32_t)i;
        ov[out + written] = make_double2(1.0, 0.0);
    }
}

hipError_t count_kept_z(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                        const FilterCtl *c, int addI, int64_t *cnt, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int wpb = 4;
    hipLaunchKernelGGL(k_count_kept_z, dim3((n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, crp,
                       cci, (const double2 *)cv, n, c, addI, cnt);
    return hipGetLastError();
}

hipError_t write_kept_z(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                        const FilterCtl *c, int addI, const int64_t *orp, int32_t *oci,
                        double *ov, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int wpb = 4;
    hipLaunchKernelGGL(k_write_kept_z, dim3((n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, crp,
                       cci, (const double2 *)cv, n, c, addI, orp, oci, (double2 *)ov);
    return hipGetLastError();
}

// C = A + B (complex values), exact zeros dropped; one thread per row.
__global__ void k_add_z(CsrView A, CsrView B, int64_t *cnt, const int64_t *crp, int32_t *cci,
                        double2 *cv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const double2 *av = (const double2 *)A.v, *bv = (const double2 *)B.v;
    int64_t p = A.rp[i], pe = A.rp[i + 1], q = B.rp[i], qe = B.rp[i + 1];
    const int64_t o = crp ? crp[i] : 0;
    int64_t k = 0;
    while (p < pe || q < qe) {
        const int ja = p < pe ? A.ci[p] : INT32_MAX;
        const int jb = q < qe ? B.ci[q] : INT32_MAX;
        int j;
        double2 s;
        if (ja == jb) {
            j = ja;
            s = make_double2(av[p].x + bv[q].x, av[p].y + bv[q].y);
            ++p;
            ++q;
        } else if (ja < jb) {
            j = ja;
            s = av[p++];
        } else {
            j = jb;
            s = bv[q++];
        }
        if (s.x == 0.0 && s.y == 0.0) continue;
        if (crp) {
            cci[o + k] = j;
            cv[o + k] = s;
        }
        k++;
    }
    if (!crp) cnt[i] = k;
}

hipError_t add_count_z(CsrView A, CsrView B, int64_t *cnt, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_z, dim3((A.n + 127) / 128), dim3(128), 0, st, A, B, cnt,
                       (const int64_t *)nullptr, (int32_t *)nullptr, (double2 *)nullptr);
    return hipGetLastError();
}

hipError_t add_write_z(CsrView A, CsrView B, const int64_t *crp, int32_t *cci, double *cv,
                       hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_z, dim3((A.n + 127) / 128), dim3(128), 0, st, A, B,
                       (int64_t *)nullptr, crp, cci, (double2 *)cv);
    return hipGetLastError();
}

// flags[0] = 1 if pattern(A) == pattern(B); flags[1] = values equal;
// flags[2] = values negated (complex values, nnz entries).
__global__ void k_compare_z(CsrView A, CsrView B, int64_t nnz, int *flags) {
    bool pat = false, eq = true, neg = true;
    const double2 *av = (const double2 *)A.v, *bv = (const double2 *)B.v;
    const int64_t m = nnz > A.n + 1 ? nnz : A.n + 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
        if (j <= A.n && A.rp[j] != B.rp[j]) pat = true;
        if (j < nnz) {
            if (A.ci[j] != B.ci[j]) pat = true;
            const double2 a = av[j], b = bv[j];
            if (a.x != b.x || a.y != b.y) eq = false;
            if (a.x != -b.x || a.y != -b.y) neg = false;
        }
    }
    const unsigned long long bp = __ballot(pat), be = __ballot(!eq), bn = __ballot(!neg);
    if (lane_id() == 0) {
        if (bp) atomicAnd(&flags[0], 0);
        if (be) atomicAnd(&flags[1], 0);
        if (bn) atomicAnd(&flags[2], 0);
    }
}

hipError_t compare_csr_z(CsrView A, CsrView B, int64_t nnz, int *flags, hipStream_t st) {
    const int64_t m = nnz > A.n + 1 ? nnz : A.n + 1;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_compare_z, dim3((unsigned)blocks), dim3(256), 0, st, A, B, nnz, flags);
    return hipGetLastError();
}

__global__ void k_identity_z(int64_t n, int64_t *rp, int32_t *ci, double2 *v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rp[i] = i;
    if (i < n) {
        ci[i] = (int32_t)i;
        v[i] = make_double2(1.0, 0.0);
    }
}

hipError_t fill_identity_z(int64_t n, int64_t *rp, int32_t *ci, double *v, hipStream_t st) {
    hipLaunchKernelGGL(k_identity_z, dim3((n + 256) / 256), dim3(256), 0, st, n, rp, ci,
                       (double2 *)v);
    return hipGetLastError();
}

// flag |= 4 if any of v[0..m) is NaN or Inf.
__global__ void k_finite(const double *v, int64_t m, int *flag) {
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride)
        bad |= !isfinite(v[j]);
    if (__ballot(bad) && lane_id() == 0) atomicOr(flag, 4);
}

hipError_t check_finite(const double *v, int64_t m, int *flag, hipStream_t st) {
    if (m == 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_finite, dim3((unsigned)blocks), dim3(256), 0, st, v, m, flag);
    return hipGetLastError();
}

// dst[q] = conj(src[pos[q]]) (complex values).
__global__ void k_gather_conj(const double2 *src, const int64_t *pos, int64_t m, double2 *dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const double2 z = src[pos[q]];
    dst[q] = make_double2(z.x, -z.y);
}

hipError_t gather_conj_z(const double *src, const int64_t *pos, int64_t m, double *dst,
                         hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_conj, dim3((m + 255) / 256), dim3(256), 0, st,
                       (const double2 *)src, pos, m, (double2 *)dst);
    return hipGetLastError();
}

}  // namespace xpm

namespace xpm {

// ============================================================== symmetric iterates
// One wave per row.  k_triu: the entries right of the diagonal (count, or
// write at orp).  k_sym_rows: row i of U^T + U, where Lt holds the
// transposed strictly upper part (its row i: columns left of i), followed
// by the entries of T on and right of the diagonal, in column order.

__global__ void k_triu(CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci, double *ov) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= T.n) return;
    int64_t k = 0;
    const int64_t o = orp ? orp[i] : 0;
    for (int64_t p0 = T.rp[i]; p0 < T.rp[i + 1]; p0 += kWave) {
        const int64_t p = p0 + lane_id();
        const bool take = p < T.rp[i + 1] && T.ci[p] > i;
        const unsigned long long m = __ballot(take);
        if (orp && take) {
            const int64_t q = o + k + __popcll(m & lanemask_lt());
            oci[q] = T.ci[p];
            ov[q] = T.v[p];
        }
        k += __popcll(m);
    }
    if (!orp && lane_id() == 0) cnt[i] = k;
}

__global__ void k_sym_rows(CsrView Lt, CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci,
                           double *ov) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= T.n) return;
    const int64_t nl = Lt.rp[i + 1] - Lt.rp[i];
    const int64_t o = orp ? orp[i] : 0;
    if (orp)
        for (int64_t q = lane_id(); q < nl; q += kWave) {
            oci[o + q] = Lt.ci[Lt.rp[i] + q];
            ov[o + q] = Lt.v[Lt.rp[i] + q];
        }
    int64_t k = nl;
    for (int64_t p0 = T.rp[i]; p0 < T.rp[i + 1]; p0 += kWave) {
        const int64_t p = p0 + lane_id();
        const bool take = p < T.rp[i + 1] && T.ci[p] >= i;
        const unsigned long long m = __ballot(take);
        if (orp && take) {
            const int64_t q = o + k + __popcll(m & lanemask_lt());
            oci[q] = T.ci[p];
            ov[q] = T.v[p];
        }
        k += __popcll(m);
    }
    if (!orp && lane_id() == 0) cnt[i] = k;
}

hipError_t triu_strict(CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci, double *ov,
                       hipStream_t st) {
    if (T.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_triu, dim3((T.n + 3) / 4), dim3(256), 0, st, T, cnt, orp, oci, ov);
    return hipGetLastError();
}

hipError_t sym_rows(CsrView Lt, CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci,
                    double *ov, hipStream_t st) {
    if (T.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sym_rows, dim3((T.n + 3) / 4), dim3(256), 0, st, Lt, T, cnt, orp, oci,
                       ov);
    return hipGetLastError();
}

}  // namespace xpm
