// Kernels of the options and diagnostics around the main path:
//  - the matrix 1-norm of H (problem (4.20) with the 1-norm),
//  - column sums of |v| of a squaring candidate, rows or tiles, for the
//    FPIM's fixed filter of section 2 (threshold eps ||T~||_1),
//  - the bandwidth l(T) of Eq. (3.1) in the caller's ordering,
//  - Y = A X, the action of a computed exponential on a dense block
//    (section 5.3's E R, Eq. (2.2)'s time step).
#include "bsr_common.hpp"

namespace xpm {

// ------------------------------------------------------------------ helpers

// Non-negative doubles order like their bit patterns: a max over them is an
// integer atomic max, independent of the order of arrival.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *dst, double x) {
    atomicMax(dst, (unsigned long long)__double_as_longlong(x));
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t m) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) p[j] = 0ull;
}

__global__ void k_fill_f64(double *p, int64_t m, double x) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) p[j] = x;
}

hipError_t fill_f64(double *p, int64_t m, double x, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, p, m, x);
    return hipGetLastError();
}

// ------------------------------------------------------------------ 1-norm
// Largest sum of |a_ij| over a row of A, each row summed in its column order
// by one thread (applied to H^T: the largest column sum of H, each column
// summed in row order).  *out (bit pattern) must start at 0.
__global__ void k_row_abs_max(CsrView A, unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < A.n)
        for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) s += fabs(A.v[p]);
    s = wave_max_f64(s);
    if (lane_id() == 0) atomic_max_nonneg(out, s);
}

hipError_t row_abs_max(CsrView A, unsigned long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out, (int64_t)1);
    if (A.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_row_abs_max, dim3((unsigned)((A.n + 255) / 256)), dim3(256), 0, st, A,
                       out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ FPIM threshold
// colsum[j] += |v| over the candidate entries of CSR rows (one wave per row).
__global__ void k_colsum_rows(const int64_t *crp, const int32_t *cci, const double *cv,
                              int64_t n, double *colsum) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    for (int64_t p = crp[i] + lane_id(); p < crp[i + 1]; p += kWave)
        atomicAdd(&colsum[cci[p]], fabs(cv[p]));
}

// The same over candidate tiles (B layout: lane l holds column l % 16 of
// rows l / 16 + 4 r): each tile adds its 16 column sums over the rows below
// n; slots past n hold zeros.
__global__ void k_colsum_tiles(int64_t n, int64_t ntiles, const int32_t *ccols,
                               const int32_t *crows, const double *ctiles, double *colsum) {
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (t >= ntiles) return;
    const int lane = lane_id();
    const d4 v = *(const d4 *)(ctiles + t * kTileElems + 4 * lane);
    double s = fabs(v[0]) + fabs(v[1]) + fabs(v[2]) + fabs(v[3]);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    const int64_t j = (int64_t)ccols[t] * kTile + (lane & 15);
    (void)crows;
    if (lane < 16 && j < n && s != 0.0) atomicAdd(&colsum[j], s);
}

// *out (bit pattern, starts at 0) = max over colsum.
__global__ void k_abs_max(const double *x, int64_t m, unsigned long long *out) {
    double s = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += (int64_t)gridDim.x * blockDim.x)
        s = fmax(s, fabs(x[j]));
    s = wave_max_f64(s);
    if (lane_id() == 0) atomic_max_nonneg(out, s);
}

// The controller takes the fixed threshold scale * max (a finished filter).
__global__ void k_theta_from_max(FilterCtl *c, const unsigned long long *mx, double scale) {
    c->eg = 0.0;
    c->theta = scale * __longlong_as_double((long long)*mx);
    c->b = 0.0;
    c->iter = 0;
    c->status = 0;
    c->done = 1;
    c->arrive = 0;
}

hipError_t fpim_theta_rows(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                           double *colsum, unsigned long long *mx, double eps, FilterCtl *c,
                           hipStream_t st) {
    hipError_t e = hipMemsetAsync(colsum, 0, sizeof(double) * (size_t)(n > 0 ? n : 1), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, mx, (int64_t)1);
    if (n > 0) {
        hipLaunchKernelGGL(k_colsum_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, crp,
                           cci, cv, n, colsum);
        hipLaunchKernelGGL(k_abs_max, dim3(1024), dim3(256), 0, st, colsum, n, mx);
    }
    hipLaunchKernelGGL(k_theta_from_max, dim3(1), dim3(1), 0, st, c, mx, eps);
    return hipGetLastError();
}

hipError_t fpim_theta_tiles(int64_t n, int64_t ntiles, const int32_t *ccols, const double *ctiles,
                            double *colsum, unsigned long long *mx, double eps, FilterCtl *c,
                            hipStream_t st) {
    hipError_t e = hipMemsetAsync(colsum, 0, sizeof(double) * (size_t)(n > 0 ? n : 1), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, mx, (int64_t)1);
    if (ntiles > 0) {
        hipLaunchKernelGGL(k_colsum_tiles, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st,
                           n, ntiles, ccols, (const int32_t *)nullptr, ctiles, colsum);
        hipLaunchKernelGGL(k_abs_max, dim3(1024), dim3(256), 0, st, colsum, n, mx);
    }
    hipLaunchKernelGGL(k_theta_from_max, dim3(1), dim3(1), 0, st, c, mx, eps);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bandwidth
// out[0] = max (j - i), out[1] = max (i - j) over the stored entries, with
// i, j the caller's indices (order[] maps the library's ordering to the
// caller's; NULL: the same).  out holds INT64_MIN before the first update.
__global__ void k_band_init(long long *out) {
    out[0] = LLONG_MIN;
    out[1] = LLONG_MIN;
}

__global__ void k_band(CsrView T, const int32_t *order, long long *out) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= T.n) return;
    const long long ri = order ? order[i] : i;
    long long up = LLONG_MIN, dn = LLONG_MIN;
    for (int64_t p = T.rp[i] + lane_id(); p < T.rp[i + 1]; p += kWave) {
        const long long cj = order ? order[T.ci[p]] : T.ci[p];
        up = max(up, cj - ri);
        dn = max(dn, ri - cj);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        up = max(up, (long long)__shfl_xor(up, o));
        dn = max(dn, (long long)__shfl_xor(dn, o));
    }
    if (lane_id() == 0 && up != LLONG_MIN) {
        atomicMax(&out[0], up);
        atomicMax(&out[1], dn);
    }
}

hipError_t band_of(CsrView T, const int32_t *order, long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_band_init, dim3(1), dim3(1), 0, st, out);
    if (T.n > 0)
        hipLaunchKernelGGL(k_band, dim3((unsigned)((T.n + 3) / 4)), dim3(256), 0, st, T, order,
                           out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ position maps
// dst[q] = src[pos[q]]  /  dst[pos[q]] += src[q]  (pos a permutation of the
// entries: each dst entry is touched once).
__global__ void k_gather_pos(const double *src, const int64_t *pos, int64_t m, double *dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) dst[q] = src[pos[q]];
}

__global__ void k_add_scatter_pos(const double *src, const int64_t *pos, int64_t m, double *dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) dst[pos[q]] += src[q];
}

hipError_t gather_pos(const double *src, const int64_t *pos, int64_t m, double *dst,
                      hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_pos, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, src, pos,
                       m, dst);
    return hipGetLastError();
}

hipError_t add_scatter_pos(const double *src, const int64_t *pos, int64_t m, double *dst,
                           hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_scatter_pos, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       src, pos, m, dst);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Y = A X
// One wave per (row i, chunk of 64 columns of X); lane = column.  The row's
// entries are read 64 at a time (one lane each) and broadcast with
// readlane; eight rows of X are loaded before their products are added, so
// each wave keeps eight loads in flight.  The products of a row are added in
// its column order, so every run gives the same bits.  The four waves of a
// workgroup take four consecutive rows with the same column chunk: they
// read largely the same rows of X, which the caches then hold.
__global__ __launch_bounds__(256) void k_spmm(CsrView A, int64_t m, const double *__restrict__ X,
                                              int64_t ldx, double *__restrict__ Y, int64_t ldy,
                                              int64_t nchunks) {
    const int lane = lane_id();
    const int64_t rows4 = (A.n + 3) / 4;
    const int64_t chunk = (int64_t)blockIdx.x / rows4;
    const int64_t i = ((int64_t)blockIdx.x % rows4) * 4 + threadIdx.x / kWave;
    if (i >= A.n || chunk >= nchunks) return;
    const int64_t c = chunk * kWave + lane;
    const bool in = c < m;
    const int64_t b = A.rp[i], e = A.rp[i + 1];
    double acc = 0.0;
    for (int64_t base = b; base < e; base += kWave) {
        const int cnt = (int)min<int64_t>(kWave, e - base);
        int myk = 0;
        double myv = 0.0;
        if (lane < cnt) {
            myk = A.ci[base + lane];
            myv = A.v[base + lane];
        }
        int j = 0;
        for (; j + 8 <= cnt; j += 8) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = __builtin_amdgcn_readlane(myk, j + u);
                x[u] = in ? X[k * ldx + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fma(readlane_f64(myv, j + u), x[u], acc);
        }
        for (; j < cnt; ++j) {
            const int64_t k = __builtin_amdgcn_readlane(myk, j);
            const double x = in ? X[k * ldx + c] : 0.0;
            acc = fma(readlane_f64(myv, j), x, acc);
        }
    }
    if (in) Y[i * ldy + c] = acc;
}

// Y = A X with A held as 16 x 16 tiles (the tile pattern of the squaring:
// tb block-row tile bases, tcols block columns, tA tiles in the A operand
// layout) on the FP64 matrix cores.  One wave per (block row I, 64 columns of
// X): four 16 x 16 output tiles, each the sum over A's tiles (I, K) of
// A_IK X_K, X_K the 16 rows of X from 16 K on (rows past n read as 0).  The
// next tile's operands load while the current tile's 16 instructions issue.
// Lane l holds X(16 K + 4 s + l / 16, c0 + 16 u + l % 16) as the B operand
// of slice s for output tile u (16 contiguous lanes read 128 contiguous
// bytes of one row of X).  The four waves of a workgroup take four
// consecutive block rows and the same columns, which read mostly the same
// rows of X.
__global__ __launch_bounds__(256) void k_spmm_tiles(int64_t n, int64_t nb, const int64_t *tb,
                                                    const int32_t *tcols,
                                                    const double *__restrict__ tA, int64_t m,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    double *__restrict__ Y, int64_t ldy,
                                                    int64_t ngroups) {
    const int lane = lane_id();
    const int64_t rows4 = (nb + 3) / 4;
    const int64_t g = (int64_t)blockIdx.x / rows4;
    const int64_t I = ((int64_t)blockIdx.x % rows4) * 4 + threadIdx.x / kWave;
    if (I >= nb || g >= ngroups) return;
    const int64_t c0 = g * 64 + (lane & 15);
    const int rsub = lane >> 4;
    d4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int64_t t, d4 &a, d4 (&b)[4]) {
        a = *(const d4 *)(tA + t * kTileElems + 4 * lane);
        const int64_t K = tcols[t];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t r = 16 * K + 4 * s + rsub;
            const bool rin = r < n;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = c0 + 16 * u;
                b[u][s] = rin && c < m ? X[r * ldx + c] : 0.0;
            }
        }
    };
    const int64_t t0 = tb[I], t1 = tb[I + 1];
    if (t0 < t1) {
        d4 a, b[4];
        load(t0, a, b);
        for (int64_t t = t0; t < t1; ++t) {
            d4 a2 = a, b2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b2[u] = b[u];
            if (t + 1 < t1) load(t + 1, a2, b2);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = mfma16(a, b[u], acc[u]);
            a = a2;
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = b2[u];
        }
    }
    // result (i, j) of tile u sits in register i / 4 of lane j + 16 (i mod 4)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = 16 * I + 4 * r + rsub;
        if (i >= n) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t c = c0 + 16 * u;
            if (c < m) Y[i * ldy + c] = acc[u][r];
        }
    }
}

hipError_t spmm_tiles(int64_t n, int64_t nb, const int64_t *tb, const int32_t *tcols,
                      const double *tA, int64_t m, const double *X, int64_t ldx, double *Y,
                      int64_t ldy, hipStream_t st) {
    if (n == 0 || m == 0) return hipSuccess;
    const int64_t ngroups = (m + 63) / 64, rows4 = (nb + 3) / 4;
    const int64_t blocks = ngroups * rows4;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_spmm_tiles, dim3((unsigned)blocks), dim3(256), 0, st, n, nb, tb, tcols,
                       tA, m, X, ldx, Y, ldy, ngroups);
    return hipGetLastError();
}

hipError_t spmm(CsrView A, int64_t m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                hipStream_t st) {
    if (A.n == 0 || m == 0) return hipSuccess;
    const int64_t nchunks = (m + kWave - 1) / kWave, rows4 = (A.n + 3) / 4;
    const int64_t blocks = nchunks * rows4;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_spmm, dim3((unsigned)blocks), dim3(256), 0, st, A, m, X, ldx, Y, ldy,
                       nchunks);
    return hipGetLastError();
}

}  // namespace xpm
