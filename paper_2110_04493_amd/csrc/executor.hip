// Host executor and C ABI of the gfx950 filtered precise-integration
// sparse exponential (Algorithm 4.2 of Wu, Zhang, Zhu, Hu, arXiv 2110.04493).
//
// The host drives a fixed sequence of kernel launches on the plan's stream
// and reads back only sizes (to allocate) and the filter controller (to know
// when Algorithm 4.1 has stopped).  All matrix data stays on the device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace xpm;
using namespace xpm::host;

namespace xpm {
namespace host {

thread_local std::string g_err;

// write_kept without the batched arguments (the signature of write_kept_z)
static hipError_t write_kept_real(const int64_t *crp, const int32_t *cci, const double *cv,
                                  int64_t n, const FilterCtl *c, int addI, const int64_t *orp,
                                  int32_t *oci, double *ov, hipStream_t st) {
    return write_kept(crp, cci, cv, n, c, addI, orp, oci, ov, st);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
}

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}


}  // namespace host
}  // namespace xpm


namespace xpm {
namespace host {

// Fixed-region mode: returns b's range to the free list, merged with its
// free neighbours.
static void arena_put(expm_plan_s &P, Buf &b) {
    if (!b.p) return;
    size_t off = (size_t)((char *)b.p - P.arena), len = b.bytes;
    auto next = P.arena_free.lower_bound(off);
    // a range that overlaps a free one was already returned (a copy of the
    // buffer released twice): keep the list as it is
    const bool overlap =
        (next != P.arena_free.end() && next->first < off + len) ||
        (next != P.arena_free.begin() && std::prev(next)->first + std::prev(next)->second > off);
    if (overlap) {
        b.p = nullptr;
        b.bytes = 0;
        return;
    }
    if (next != P.arena_free.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            P.arena_free.erase(prev);
        }
    }
    if (next != P.arena_free.end() && off + len == next->first) {
        len += next->second;
        P.arena_free.erase(next);
    }
    P.arena_free[off] = len;
    P.live -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

// Fixed-region mode: b becomes a range of at least `bytes` bytes (the first
// free range that holds it); its old contents are not kept, as with the
// pool.
static int arena_grow(expm_plan_s &P, Buf &b, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    arena_put(P, b);
    for (auto it = P.arena_free.begin(); it != P.arena_free.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, rest = it->second - bytes;
        P.arena_free.erase(it);
        if (rest) P.arena_free[off + bytes] = rest;
        b.p = P.arena + off;
        b.bytes = bytes;
        P.live += bytes;
        P.peak = std::max(P.peak, P.live);
        return EXPM_OK;
    }
    return fail(EXPM_ENOMEM,
                "the %zu-byte static scratch of expm_sparse_noalloc is exhausted (no free range "
                "of %zu bytes with %zu bytes in use)", P.arena_bytes, bytes, P.live);
}

int ensure(expm_plan_s &P, Buf &b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return EXPM_OK;
    if (P.arena) return arena_grow(P, b, bytes);
    if (b.p) {
        HIPCHK(hipFreeAsync(b.p, P.st));
        P.live -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 255) & ~(size_t)255;
    hipError_t e = hipMallocAsync(&b.p, want, P.st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        e = hipMallocAsync(&b.p, bytes, P.st);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(EXPM_ENOMEM, "cannot allocate %zu bytes of device workspace", bytes);
    }
    b.bytes = want;
    P.live += want;
    P.peak = std::max(P.peak, P.live);
    return EXPM_OK;
}

// Buffers that trade places between roles (iterates and checkpoints, tile
// sets) are grown to the largest size their roles need, once, so that
// later calls allocate nothing: b is grown to ref's capacity when smaller.
int reserve_as(expm_plan_s &P, Buf &b, const Buf &ref) {
    if (b.bytes >= ref.bytes || ref.bytes == 0) return EXPM_OK;
    if (P.arena) return arena_grow(P, b, ref.bytes);
    if (b.p) {
        HIPCHK(hipFreeAsync(b.p, P.st));
        P.live -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (hipMallocAsync(&b.p, ref.bytes, P.st) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(EXPM_ENOMEM, "cannot allocate %zu bytes of device workspace", ref.bytes);
    }
    b.bytes = ref.bytes;
    P.live += b.bytes;
    P.peak = std::max(P.peak, P.live);
    return EXPM_OK;
}

int reserve_as(expm_plan_s &P, DCsr &d, const DCsr &ref) {
    CHK(reserve_as(P, d.rp, ref.rp));
    CHK(reserve_as(P, d.ci, ref.ci));
    return reserve_as(P, d.v, ref.v);
}

int reserve_as(expm_plan_s &P, TileSet &t, const TileSet &ref) {
    Buf *a[] = {&t.lo, &t.words, &t.woff, &t.rt,   &t.cnt, &t.tb,
                &t.tA, &t.tB,    &t.cols, &t.rows, &t.seg, &t.mir};
    const Buf *r[] = {&ref.lo, &ref.words, &ref.woff, &ref.rt,   &ref.cnt, &ref.tb,
                      &ref.tA, &ref.tB,    &ref.cols, &ref.rows, &ref.seg, &ref.mir};
    for (int j = 0; j < 12; ++j) CHK(reserve_as(P, *a[j], *r[j]));
    return EXPM_OK;
}

void release(expm_plan_s &P, Buf &b) {
    if (b.p && P.arena) {
        arena_put(P, b);
    } else if (b.p) {
        (void)hipFreeAsync(b.p, P.st);
        P.live -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

void release(expm_plan_s &P, DCsr &A) {
    release(P, A.rp);
    release(P, A.ci);
    release(P, A.v);
    A.n = A.nnz = 0;
}

int ensure_csr(expm_plan_s &P, DCsr &A, int64_t n, int64_t nnz, int vw) {
    CHK(ensure(P, A.rp, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, A.ci, sizeof(int32_t) * nnz));
    CHK(ensure(P, A.v, sizeof(double) * vw * nnz));
    A.n = n;
    A.nnz = nnz;
    return EXPM_OK;
}

// Copy of a device CSR (checkpoints, Taylor terms) into dst's buffers,
// grown when too small.
int copy_csr(expm_plan_s &P, DCsr &dst, const DCsr &src, int vw) {
    CHK(ensure_csr(P, dst, src.n, src.nnz, vw));
    HIPCHK(hipMemcpyAsync(dst.rp.p, src.rp.p, sizeof(int64_t) * (src.n + 1),
                          hipMemcpyDeviceToDevice, P.st));
    if (src.nnz) {
        HIPCHK(hipMemcpyAsync(dst.ci.p, src.ci.p, sizeof(int32_t) * src.nnz,
                              hipMemcpyDeviceToDevice, P.st));
        HIPCHK(hipMemcpyAsync(dst.v.p, src.v.p, sizeof(double) * vw * src.nnz,
                              hipMemcpyDeviceToDevice, P.st));
    }
    return EXPM_OK;
}

DCsr &push_reuse(std::vector<DCsr> &live, std::vector<DCsr> &pool) {
    live.emplace_back();
    if (!pool.empty()) {
        live.back() = pool.back();
        pool.pop_back();
    }
    return live.back();
}

void retire(std::vector<DCsr> &live, std::vector<DCsr> &pool) {
    // reversed, so that push_reuse hands entry i its own buffers back
    for (auto it = live.rbegin(); it != live.rend(); ++it) pool.push_back(*it);
    live.clear();
}

int sync(expm_plan_s &P) {
    HIPCHK(hipStreamSynchronize(P.st));
    return EXPM_OK;
}

int scan(expm_plan_s &P, const int64_t *in, int64_t *out, int64_t n) {
    size_t tb = scan_tmp_bytes(n);
    CHK(ensure(P, P.scan_tmp, tb));
    HIPCHK(scan_i64(in, out, n, P.scan_tmp.p, P.scan_tmp.bytes, P.st));
    return EXPM_OK;
}

void *out_alloc(expm_plan_s &P, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (P.arena) return nullptr;   // outputs come from alloc_output only
    void *p = nullptr;
    if (P.opts.allocator && P.opts.allocator->alloc) {
        p = P.opts.allocator->alloc(bytes, P.st, P.opts.allocator->ctx);
    } else if (hipMallocAsync(&p, bytes, P.st) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) P.outputs.push_back(p);
    return p;
}

void out_free(expm_plan_s &P, void *p) {
    if (!p || P.arena) return;   // fixed-region outputs belong to the caller
    auto it = std::find(P.outputs.begin(), P.outputs.end(), p);
    if (it == P.outputs.end()) return;
    P.outputs.erase(it);
    if (P.opts.allocator && P.opts.allocator->free)
        P.opts.allocator->free(p, P.st, P.opts.allocator->ctx);
    else
        (void)hipFreeAsync(p, P.st);
}

int alloc_output(expm_plan_s &P, int64_t n, int64_t nnz, int64_t **rp, int32_t **ci,
                 double **v, int vw) {
    if (P.arena) {
        P.na_need = nnz;
        if (nnz > P.na_cap)
            return fail(EXPM_ENOMEM, "the output holds %lld entries, more than the %lld the "
                        "caller's buffers take", (long long)nnz, (long long)P.na_cap);
        *rp = P.na_rp;
        *ci = P.na_ci;
        *v = P.na_v;
        return EXPM_OK;
    }
    *rp = (int64_t *)out_alloc(P, sizeof(int64_t) * (n + 1));
    *ci = (int32_t *)out_alloc(P, sizeof(int32_t) * nnz);
    *v = (double *)out_alloc(P, sizeof(double) * vw * nnz);
    if (!*rp || !*ci || !*v) {
        out_free(P, *rp);
        out_free(P, *ci);
        out_free(P, *v);
        *rp = nullptr;
        *ci = nullptr;
        *v = nullptr;
        return fail(EXPM_ENOMEM, "cannot allocate the output (%lld entries)", (long long)nnz);
    }
    return EXPM_OK;
}

// ------------------------------------------------------------------ planner
// Eq. (4.5): r0(M, x) = sum_{k>=0} x^{M+1+k} / (M! k! (M+1+k)), all terms
// positive; stop once a term no longer changes the sum at 2^-60.
double plan_r0(int M, double x) {
    if (!(x > 0.0)) return 0.0;
    double lead = x;                      // x^{M+1} / M!
    for (int j = 1; j <= M; ++j) lead *= x / (double)j;
    double total = 0.0, pk = lead;
    for (int k = 0;; ++k) {
        if (k) pk *= x / (double)k;
        const double t = pk / (double)(M + 1 + k);
        total += t;
        if (t < ldexp(total, -60) || k > 100000) break;
    }
    return total;
}

// Problem (4.20) by enumeration: N in [N0, N0 + 50], the least M >= 1 meeting
// the tolerance for each N, minimal M 2^N, first (smallest N) on ties.
int plan_mn(double nh, double eps, int *Mo, int *No) {
    if (!(nh >= 0.0) || !isfinite(nh) || !(eps > 0.0)) return EXPM_EINVAL;
    int n0 = 0;
    if (nh > 1.0) n0 = (int)ceil(log2(nh));
    while (ldexp(nh, -n0) > 1.0) ++n0;
    int bestM = 0, bestN = 0;
    double bestCost = 0.0;
    for (int N = n0; N <= n0 + 50; ++N) {
        const double x = ldexp(nh, -N);
        int M = 1;
        while (M <= 170 && ldexp(plan_r0(M, x), N) > eps) ++M;
        if (M > 170) continue;
        const double cost = ldexp((double)M, N);
        if (bestM == 0 || cost < bestCost) {
            bestM = M;
            bestN = N;
            bestCost = cost;
        }
    }
    if (bestM == 0) return EXPM_ERANGE;
    *Mo = bestM;
    *No = bestN;
    return EXPM_OK;
}

// ------------------------------------------------------------------ SpGEMM driver
// C = alphaA * A + A * B (divided by div), into the candidate buffers
// (P.crp, P.cci, P.cv).  Returns the candidate total in *total; with rowsq
// the per-row sums of (c + delta)^2 are left in P.rowsq.
int spgemm(expm_plan_s &P, CsrView A, int64_t nnzA, CsrView B, double alphaA, double div, bool rowsq,
           int64_t *total, bool cplx) {
    const int64_t n = A.n;
    hipStream_t st = P.st;
    CHK(ensure(P, P.lo, sizeof(int32_t) * n));
    CHK(ensure(P, P.words, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.woff, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.ub, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.crp, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.sbytes, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.soff, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.lists, sizeof(int32_t) * (size_t)kNumClasses * (n > 0 ? n : 1)));
    CHK(ensure(P, P.counts, sizeof(int) * 16));
    int64_t *words = (int64_t *)P.words.p, *woff = (int64_t *)P.woff.p;
    const bool prof = P.opts.profile == 1 && P.have_events;
    if (prof) HIPCHK(hipEventRecord(P.ev[0], st));
    HIPCHK(row_bounds(A, B, alphaA != 0.0, (int32_t *)P.lo.p, words, (int64_t *)P.ub.p, st));
    CHK(scan(P, words, woff, n));
    HIPCHK(bin_rows(woff, nullptr, n, 0, (int *)P.counts.p, (int32_t *)P.lists.p, st));
    int64_t *hl = (int64_t *)P.host;
    HIPCHK(hipMemcpyAsync(hl, woff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hl + 1, P.counts.p, sizeof(int) * kSymClasses, hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    const int64_t twords = hl[0];
    int symc[kSymClasses];
    memcpy(symc, hl + 1, sizeof symc);
    CHK(ensure(P, P.bitmaps, sizeof(uint32_t) * twords));
    int64_t *cnt = (int64_t *)P.cnt.p, *crp = (int64_t *)P.crp.p;
    HIPCHK(symbolic(A, B, alphaA != 0.0, (const int32_t *)P.lo.p, woff, (uint32_t *)P.bitmaps.p,
                    cnt, symc, (const int32_t *)P.lists.p, n, st));
    CHK(scan(P, cnt, crp, n));
    HIPCHK(numeric_scratch_sizes(woff, crp, n, (int64_t *)P.sbytes.p, st, cplx));
    CHK(scan(P, (const int64_t *)P.sbytes.p, (int64_t *)P.soff.p, n));
    HIPCHK(bin_rows(woff, crp, n, cplx ? 2 : 1, (int *)P.counts.p, (int32_t *)P.lists.p, st));
    if (prof) {
        // partial products = sum of ub minus the rows of the alphaA*A term
        CHK(ensure(P, P.tmp1, sizeof(int64_t) * (n + 1)));
        CHK(scan(P, (const int64_t *)P.ub.p, (int64_t *)P.tmp1.p, n));
        HIPCHK(hipMemcpyAsync(hl + 8, (int64_t *)P.tmp1.p + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(hl, crp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hl + 1, (int64_t *)P.soff.p + n, sizeof(int64_t),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hl + 2, P.counts.p, sizeof(int) * kNumClasses, hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    const int64_t cand = hl[0], gscratch = hl[1];
    int numc[kNumClasses];
    memcpy(numc, hl + 2, sizeof numc);
    CHK(ensure(P, P.cci, sizeof(int32_t) * cand));
    CHK(ensure(P, P.cv, sizeof(double) * (cplx ? 2 : 1) * cand));
    if (gscratch) CHK(ensure(P, P.scratch, (size_t)gscratch));
    if (rowsq) CHK(ensure(P, P.rowsq, sizeof(double) * (n + 1)));
    if (prof) {
        int64_t ubt;
        memcpy(&ubt, hl + 8, sizeof ubt);
        P.last_fma = alphaA != 0.0 ? ubt - nnzA : ubt;
        HIPCHK(hipEventRecord(P.ev[1], st));
    }
    HIPCHK((cplx ? numeric_z : numeric)(A, B, alphaA, div, (const int32_t *)P.lo.p, woff,
                                        (const uint32_t *)P.bitmaps.p, crp, (int32_t *)P.cci.p,
                                        (double *)P.cv.p, rowsq ? (double *)P.rowsq.p : nullptr,
                                        numc, (const int32_t *)P.lists.p, n, P.scratch.p,
                                        (const int64_t *)P.soff.p, st));
    if (prof) HIPCHK(hipEventRecord(P.ev[2], st));
    *total = cand;
    return EXPM_OK;
}


// Algorithm 4.1 on the candidate values plus the row counts of the kept
// entries: leaves the threshold in P.ctl, kept counts scanned into P.krp.
// norm2 (device) scales eg for the relative squaring budget; theta_fixed >= 0
// (or -1 to keep everything) skips the search.
int filter_and_count(expm_plan_s &P, int64_t n, int64_t cand, double eg_scale,
                     const double *norm2, bool use_fixed, double theta_fixed, bool addI,
                     FilterCtl *hctl, int64_t *kept, bool cplx) {
    hipStream_t st = P.st;
    CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    FilterCtl *ctl = (FilterCtl *)P.ctl.p;
    if (use_fixed && theta_fixed != kThetaOnDevice)
        HIPCHK(filter_init_theta(ctl, theta_fixed, st));
    else if (!use_fixed)
        HIPCHK(filter_init(ctl, eg_scale, norm2, P.opts.e_r, P.opts.max_filter_iter, st));
    const int64_t *crp = (const int64_t *)P.crp.p;
    for (int round = 0;; ++round) {
        if (!use_fixed) {
            for (int j = 0; j < 4; ++j)
                HIPCHK((cplx ? filter_pass_z : filter_pass)((const double *)P.cv.p, crp + n, cand,
                                                            ctl, (double *)P.part.p, kParts, st));
        }
        if (cplx)
            HIPCHK(count_kept_z(crp, (const int32_t *)P.cci.p, (const double *)P.cv.p, n, ctl,
                                addI ? 1 : 0, (int64_t *)P.cnt.p, st));
        else
            HIPCHK(count_kept(crp, (const int32_t *)P.cci.p, (const double *)P.cv.p, n, ctl,
                              addI ? 1 : 0, (int64_t *)P.cnt.p, st));
        CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.krp.p, n));
        HIPCHK(hipMemcpyAsync(P.host, ctl, sizeof(FilterCtl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync((char *)P.host + 256, (int64_t *)P.krp.p + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        memcpy(hctl, P.host, sizeof(FilterCtl));
        memcpy(kept, (char *)P.host + 256, sizeof(int64_t));
        if (hctl->done) break;
        if (round > P.opts.max_filter_iter)
            return fail(EXPM_ENOTCONV, "Algorithm 4.1 did not stop");
    }
    if (hctl->status)
        return fail(EXPM_ENOTCONV, "Algorithm 4.1 reached %d iterations (budget %g)",
                    hctl->iter, hctl->eg);
    return EXPM_OK;
}

// Writes the kept candidate entries (rows from P.krp) into dst (capacity
// must hold `kept` entries; dst.rp receives P.krp).
int write_filtered(expm_plan_s &P, int64_t n, DCsr &dst, int64_t kept, bool addI,
                   bool exact_alloc, bool cplx) {
    if (exact_alloc) release(P, dst);
    CHK(ensure_csr(P, dst, n, kept, cplx ? 2 : 1));
    HIPCHK(hipMemcpyAsync(dst.rp.p, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                          P.st));
    HIPCHK((cplx ? write_kept_z : write_kept_real)(
        (const int64_t *)P.crp.p, (const int32_t *)P.cci.p, (const double *)P.cv.p, n,
        (const FilterCtl *)P.ctl.p, addI ? 1 : 0, (const int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
        (double *)dst.v.p, P.st));
    return EXPM_OK;
}

// dst = A + B with exact zeros dropped (capacity nnz(A) + nnz(B)).
int sparse_add(expm_plan_s &P, const DCsr &A, const DCsr &B, DCsr &dst) {
    const int64_t n = A.n;
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure_csr(P, dst, n, A.nnz + B.nnz));
    HIPCHK(add_count(A.view(), B.view(), (int64_t *)P.cnt.p, P.st));
    CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)dst.rp.p, n));
    HIPCHK(add_write(A.view(), B.view(), (const int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
                     (double *)dst.v.p, P.st));
    return EXPM_OK;
}

// dst = sum of the Taylor terms P.taylor in order (exact zeros removed): one
// multi-term pass (rows too wide for LDS in global scratch), or, past
// kSumMaxTerms terms, the terms added pairwise (the same sums in the same
// order).
int sum_taylor(expm_plan_s &P, DCsr &dst) {
    const int m = (int)P.taylor.size();
    const int64_t n = P.taylor[0].n;
    if (m == 1) return copy_csr(P, dst, P.taylor[0]);
    if (m <= kSumMaxTerms) {
        SumTerms T{};
        for (int t = 0; t < m; ++t) {
            T.rp[t] = (const int64_t *)P.taylor[t].rp.p;
            T.ci[t] = (const int32_t *)P.taylor[t].ci.p;
            T.v[t] = (const double *)P.taylor[t].v.p;
        }
        T.m = m;
        CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.tmp1, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.tmp2, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.flags, sizeof(int) * 4));
        // global scratch of the rows too wide for LDS
        int64_t *bytes = (int64_t *)P.tmp1.p, *goff = (int64_t *)P.tmp2.p;
        HIPCHK(sum_terms_bounds(T, n, bytes, P.st));
        CHK(scan(P, bytes, goff, n));
        int64_t *hl = (int64_t *)P.host;
        HIPCHK(hipMemcpyAsync(hl, goff + n, sizeof(int64_t), hipMemcpyDeviceToHost, P.st));
        CHK(sync(P));
        CHK(ensure(P, P.scratch, (size_t)hl[0] + 256));
        char *gscr = (char *)P.scratch.p;
        HIPCHK(hipMemsetAsync(P.flags.p, 0, sizeof(int), P.st));
        HIPCHK(sum_terms_count(T, n, gscr, goff, (int64_t *)P.cnt.p, (int *)P.flags.p, P.st));
        CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.krp.p, n));
        HIPCHK(hipMemcpyAsync(hl, (int64_t *)P.krp.p + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, P.st));
        HIPCHK(hipMemcpyAsync(hl + 1, P.flags.p, sizeof(int), hipMemcpyDeviceToHost, P.st));
        CHK(sync(P));
        const int64_t nnz = hl[0];
        if ((int)(hl[1] & 0xffffffff))
            return fail(EXPM_EHIP, "Taylor sum: a row exceeded its working memory");
        CHK(ensure_csr(P, dst, n, nnz));
        HIPCHK(hipMemcpyAsync(dst.rp.p, P.krp.p, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToDevice, P.st));
        HIPCHK(sum_terms_write(T, n, gscr, goff, (const int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
                               (double *)dst.v.p, P.st));
        return EXPM_OK;
    }
    CHK(copy_csr(P, dst, P.taylor[0]));
    for (int t = 1; t < m; ++t) {
        CHK(sparse_add(P, dst, P.taylor[t], P.Tnew));
        std::swap(dst, P.Tnew);
    }
    return EXPM_OK;
}

// Device transpose of A into dst.
int transpose_csr(expm_plan_s &P, const DCsr &A, DCsr &dst) {
    const int64_t n = A.n;
    CHK(ensure_csr(P, dst, n, A.nnz));
    CHK(ensure(P, P.tmp1, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.tmp2, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cci, sizeof(int32_t) * A.nnz));
    CHK(ensure(P, P.cv, sizeof(double) * A.nnz));
    CHK(ensure(P, P.scan_tmp, scan_tmp_bytes(n)));
    HIPCHK(transpose(A.view(), A.nnz, (int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
                     (double *)dst.v.p, (int64_t *)P.tmp1.p, (int64_t *)P.tmp2.p,
                     (int32_t *)P.cci.p, (double *)P.cv.p, P.scan_tmp.p, P.scan_tmp.bytes,
                     P.st));
    return EXPM_OK;
}

// dst: A's transposed pattern; its value array holds, for every entry, the
// position (int64) of the same entry in A.
int transpose_pos(expm_plan_s &P, const DCsr &A, DCsr &dst) {
    const int64_t n = A.n;
    CHK(ensure_csr(P, dst, n, A.nnz));
    CHK(ensure(P, P.tmp1, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.tmp2, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cci, sizeof(int32_t) * A.nnz));
    CHK(ensure(P, P.cv, sizeof(int64_t) * A.nnz));
    CHK(ensure(P, P.scan_tmp, scan_tmp_bytes(n)));
    HIPCHK(transpose_index(A.view(), A.nnz, (int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
                           (int64_t *)dst.v.p, (int64_t *)P.tmp1.p, (int64_t *)P.tmp2.p,
                           (int32_t *)P.cci.p, (int64_t *)P.cv.p, P.scan_tmp.p,
                           P.scan_tmp.bytes, P.st));
    return EXPM_OK;
}

// Masked products on the mask's pattern (see masked_products).  The scratch
// for rows whose working set exceeds LDS is sized by a first call and the
// call is repeated once with enough room.
int masked(expm_plan_s &P, CsrView M, CsrView D, double gamma, MaskTerm t1, MaskTerm t2,
           double div, double *out) {
    const int64_t n = M.n;
    CHK(ensure(P, P.scratch, masked_meta_bytes(n)));
    size_t need = 0;
    hipError_t e = masked_products(M, D, gamma, t1, t2, div, out, P.scratch.p, P.scratch.bytes,
                                   &need, P.st);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        CHK(sync(P));
        CHK(ensure(P, P.scratch, need));
        e = masked_products(M, D, gamma, t1, t2, div, out, P.scratch.p, P.scratch.bytes, &need,
                            P.st);
    }
    HIPCHK(e);
    return EXPM_OK;
}

CsrView empty_view() { return CsrView{0, nullptr, nullptr, nullptr}; }

// ------------------------------------------------------------------ forward

int check_view(const expm_csr_cview *H) {
    if (!H) return fail(EXPM_EINVAL, "H is NULL");
    if (H->n < 0 || H->n > INT32_MAX - 1) return fail(EXPM_EINVAL, "n = %lld out of range",
                                                      (long long)H->n);
    if (H->nnz < 0) return fail(EXPM_EINVAL, "nnz < 0");
    if (H->n > 0 && !H->rowptr) return fail(EXPM_EINVAL, "rowptr is NULL");
    if (H->nnz > 0 && (!H->col || !H->val)) return fail(EXPM_EINVAL, "col/val is NULL");
    return EXPM_OK;
}

int output_identity(expm_plan_s &P, int64_t n, expm_csr *E) {
    int64_t *rp;
    int32_t *ci;
    double *v;
    CHK(alloc_output(P, n, n, &rp, &ci, &v));
    HIPCHK(fill_identity(n, rp, ci, v, P.st));
    E->n = n;
    E->nnz = n;
    E->rowptr = rp;
    E->col = ci;
    E->val = v;
    return EXPM_OK;
}

// Is H normal?  Exact symmetric / skew-symmetric, else the commutator test.
int detect_normal(expm_plan_s &P, const DCsr &H, double nh, int *normal) {
    const int64_t n = H.n;
    DCsr Ht;
    CHK(transpose_csr(P, H, Ht));
    CHK(ensure(P, P.flags, sizeof(int) * 4));
    int ones[3] = {1, 1, 1};
    HIPCHK(hipMemcpyAsync(P.flags.p, ones, sizeof ones, hipMemcpyHostToDevice, P.st));
    HIPCHK(compare_csr(H.view(), Ht.view(), H.nnz, (int *)P.flags.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.flags.p, sizeof(int) * 3, hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    int f[3];
    memcpy(f, P.host, sizeof f);
    P.last_sym = f[0] && f[1];
    if (f[0] && (f[1] || f[2])) {
        *normal = 1;
        release(P, Ht);
        return EXPM_OK;
    }
    // ||H H^T - H^T H||_F <= 16 u ||H||_F^2
    int64_t c1, c2;
    CHK(spgemm(P, H.view(), H.nnz, Ht.view(), 0.0, 1.0, false, &c1));
    DCsr X, Y;
    CHK(ensure_csr(P, X, n, c1));
    HIPCHK(hipMemcpyAsync(X.rp.p, P.crp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, P.st));
    HIPCHK(hipMemcpyAsync(X.ci.p, P.cci.p, sizeof(int32_t) * c1, hipMemcpyDeviceToDevice, P.st));
    HIPCHK(hipMemcpyAsync(X.v.p, P.cv.p, sizeof(double) * c1, hipMemcpyDeviceToDevice, P.st));
    CHK(spgemm(P, Ht.view(), Ht.nnz, H.view(), 0.0, 1.0, false, &c2));
    CHK(ensure_csr(P, Y, n, c2));
    HIPCHK(hipMemcpyAsync(Y.rp.p, P.crp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, P.st));
    HIPCHK(hipMemcpyAsync(Y.ci.p, P.cci.p, sizeof(int32_t) * c2, hipMemcpyDeviceToDevice, P.st));
    HIPCHK(scale_ldexp((const double *)P.cv.p, (double *)Y.v.p, c2, 0, P.st));
    // Z = H H^T - H^T H
    DCsr Z;
    HIPCHK(negate_values((double *)Y.v.p, c2, P.st));
    CHK(sparse_add(P, X, Y, Z));
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    HIPCHK(sumsq((const double *)Z.v.p, (const int64_t *)Z.rp.p + n, Z.nnz, (double *)P.part.p,
                 kParts, (double *)P.norm2.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.norm2.p, sizeof(double), hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    double c2n;
    memcpy(&c2n, P.host, sizeof c2n);
    *normal = sqrt(c2n) <= 16.0 * ldexp(1.0, -53) * nh * nh;
    release(P, Ht);
    release(P, X);
    release(P, Y);
    release(P, Z);
    return EXPM_OK;
}

// Is H exactly symmetric (pattern and values)?
int exact_symmetry(expm_plan_s &P, const DCsr &H, int *sym) {
    DCsr Ht;
    auto free_ht = at_exit([&] { release(P, Ht); });
    CHK(transpose_csr(P, H, Ht));
    CHK(ensure(P, P.flags, sizeof(int) * 4));
    const int ones[3] = {1, 1, 1};
    HIPCHK(hipMemcpyAsync(P.flags.p, ones, sizeof ones, hipMemcpyHostToDevice, P.st));
    HIPCHK(compare_csr(H.view(), Ht.view(), H.nnz, (int *)P.flags.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.flags.p, sizeof(int) * 3, hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    int f[3];
    memcpy(f, P.host, sizeof f);
    *sym = f[0] && f[1];
    return EXPM_OK;
}

// T <- U + U^T for U the part of T on and right of the diagonal: an exactly
// symmetric T_0 for symmetric H (the Taylor terms are symmetric up to
// rounding only).  Uses P.S, P.Snew and P.Tnew as workspace.
int symmetrize_upper(expm_plan_s &P, DCsr &T) {
    const int64_t n = T.n;
    hipStream_t st = P.st;
    DCsr &Su = P.S, &Lt = P.Snew, &Tn = P.Tnew;
    CHK(ensure(P, P.sym_cnt, sizeof(int64_t) * (n + 1)));
    int64_t *cnt = (int64_t *)P.sym_cnt.p;
    int64_t *hl = (int64_t *)P.host;
    // the strictly upper part
    CHK(ensure(P, Su.rp, sizeof(int64_t) * (n + 1)));
    HIPCHK(triu_strict(T.view(), cnt, nullptr, nullptr, nullptr, st));
    CHK(scan(P, cnt, (int64_t *)Su.rp.p, n));
    HIPCHK(hipMemcpyAsync(hl, (int64_t *)Su.rp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    const int64_t nu = hl[0];
    CHK(ensure_csr(P, Su, n, nu));
    HIPCHK(triu_strict(T.view(), nullptr, (const int64_t *)Su.rp.p, (int32_t *)Su.ci.p,
                       (double *)Su.v.p, st));
    // its transpose, then U^T's rows followed by U's
    CHK(transpose_csr(P, Su, Lt));
    HIPCHK(sym_rows(Lt.view(), T.view(), cnt, nullptr, nullptr, nullptr, st));
    CHK(ensure(P, Tn.rp, sizeof(int64_t) * (n + 1)));
    CHK(scan(P, cnt, (int64_t *)Tn.rp.p, n));
    HIPCHK(hipMemcpyAsync(hl, (int64_t *)Tn.rp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    const int64_t m = hl[0];
    CHK(ensure_csr(P, Tn, n, m));
    HIPCHK(sym_rows(Lt.view(), T.view(), nullptr, (const int64_t *)Tn.rp.p, (int32_t *)Tn.ci.p,
                    (double *)Tn.v.p, st));
    std::swap(T, Tn);
    T.nnz = m;
    return EXPM_OK;
}

// Forgets the state of the last forward; the buffers stay with the plan
// for the next call (expm_free releases them).
void free_adjoint_state(expm_plan_s &P) {
    retire(P.taylor, P.taylor_pool);
    retire(P.ckpt, P.ckpt_pool);
    P.ckpt_at.clear();
    P.sq_path.clear();
    P.TN.nnz = 0;
    P.Epat.nnz = 0;
    P.theta.clear();
    P.have_fwd = false;
}

// One filtered squaring T <- filter(2T + T*T) into dst; with theta_fixed the
// stored threshold replaces the search.  Fills the step's statistics when
// stat_i > 0.  addI: dst = I + filtered (the finish step), exact_alloc: dst
// gets exactly the kept entries.
// Tiles need a block-row bit map in LDS (at most n / 512 words) and are
// switched off entirely by a fill threshold above 1.
bool tiles_allowed(const expm_plan_s &P, int64_t n) {
    return P.bsr_min_fill <= 1.0 && bsr_lds_words(n) * 4 <= 65536;
}

int square_step(expm_plan_s &P, const DCsr &T, DCsr &dst, double a_ri, bool use_fixed,
                double theta_fixed, bool addI, bool exact_alloc, int stat_i, int step) {
    const int64_t n = T.n;
    // Tile or scalar product: decided once per squaring step from the tile
    // fill of T and recorded, so that recomputation repeats the same path.
    bool tiles = false;
    bool have_pattern = false;
    if (step >= 1 && (int)P.sq_path.size() >= step) {
        tiles = P.sq_path[step - 1] != 0;
    } else {
        if (!addI && tiles_allowed(P, n)) {
            double fill = 0.0;
            // once a step has run on tiles the next ones will too (the fill
            // grows with the band): take the product's pattern counts along
            const bool likely = !P.sq_path.empty() && P.sq_path.back() != 0;
            CHK(bsr_pattern(P, T.view(), T.nnz, P.tsT, &fill, likely));
            have_pattern = true;
            tiles = P.tsT.ntiles > 0 && P.tsT.ntiles < INT32_MAX && fill >= P.bsr_min_fill;
        }
        if (step >= 1) P.sq_path.push_back(tiles ? 1 : 0);
    }
    if (stat_i > 0 && stat_i < EXPM_MAXSTEP && !tiles) P.stats.sq_tiles[stat_i] = 0;
    if (!tiles) P.c_pre = false;
    if (tiles) {
        if (!have_pattern) {
            double fill;
            CHK(bsr_pattern(P, T.view(), T.nnz, P.tsT, &fill, true));
        }
        return square_step_bsr(P, T, dst, a_ri, use_fixed, theta_fixed, exact_alloc, stat_i);
    }
    int64_t cand;
    // the FPIM's filter (forward steps): a threshold from the candidate's
    // 1-norm instead of Algorithm 4.1
    const bool fpim = P.fpim_eps > 0.0 && !use_fixed;
    CHK(spgemm(P, T.view(), T.nnz, T.view(), 2.0, 1.0, !use_fixed && !fpim, &cand));
    if (fpim) {
        CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
        CHK(ensure(P, P.colsum, sizeof(double) * (n + 1)));
        CHK(ensure(P, P.amax, sizeof(unsigned long long) * 2));
        HIPCHK(fpim_theta_rows((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                               (const double *)P.cv.p, n, (double *)P.colsum.p,
                               (unsigned long long *)P.amax.p, P.fpim_eps, (FilterCtl *)P.ctl.p,
                               P.st));
        use_fixed = true;
        theta_fixed = kThetaOnDevice;
    } else if (!use_fixed) {
        CHK(ensure(P, P.norm2, sizeof(double) * 2));
        CHK(ensure(P, P.part, sizeof(double) * kParts));
        HIPCHK(sum_values((const double *)P.rowsq.p, n, (double *)P.part.p, kParts,
                          (double *)P.norm2.p, P.st));
    }
    FilterCtl h{};
    int64_t kept;
    CHK(filter_and_count(P, n, cand, a_ri, (const double *)P.norm2.p, use_fixed, theta_fixed,
                         addI, &h, &kept));
    CHK(write_filtered(P, n, dst, kept, addI, exact_alloc));
    if (stat_i > 0 && stat_i < EXPM_MAXSTEP && P.opts.profile == 1 && P.have_events) {
        HIPCHK(hipEventRecord(P.ev[3], P.st));
        HIPCHK(hipEventSynchronize(P.ev[3]));
        float t0, t1, t2;
        HIPCHK(hipEventElapsedTime(&t0, P.ev[0], P.ev[1]));
        HIPCHK(hipEventElapsedTime(&t1, P.ev[1], P.ev[2]));
        HIPCHK(hipEventElapsedTime(&t2, P.ev[2], P.ev[3]));
        P.stats.t_sym_ms[stat_i] = t0;
        P.stats.t_num_ms[stat_i] = t1;
        P.stats.t_filter_ms[stat_i] = t2;
        P.stats.sq_fma[stat_i] = P.last_fma;
        P.stats.sq_in[stat_i] = T.nnz;
    }
    if (stat_i > 0 && stat_i < EXPM_MAXSTEP) {
        expm_stats &S = P.stats;
        S.sq_theta[stat_i] = h.theta;
        S.sq_iters[stat_i] = h.iter;
        S.sq_cand[stat_i] = cand;
        S.sq_kept[stat_i] = kept;
        S.sq_budget[stat_i] = fpim ? h.theta : h.eg;
        S.sq_normF[stat_i] = a_ri > 0 && !fpim ? h.eg / a_ri : 0.0;
        S.sq_dropped[stat_i] = h.b;
    }
    return EXPM_OK;
}

// Algorithm 4.2 steps 1-3 on H: copies H into dst (from host memory when
// the view says so), validates it, computes ||H||_F and the norm of
// opts.norm on the device, then (M, N) by problem (4.20), the normality and
// a, r0 and eg0.  A zero H gives M = N = 0 and norm_fro = 0.
int plan_input(expm_plan_s &P, const expm_csr_cview *Hv, double eps, DCsr &dst,
               expm_analysis *A) {
    hipStream_t st = P.st;
    const int64_t n = Hv->n, nnz = Hv->nnz;
    memset(A, 0, sizeof *A);
    A->n = n;
    A->nnz = nnz;
    const hipMemcpyKind kind = Hv->on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CHK(ensure_csr(P, dst, n, nnz));
    HIPCHK(hipMemcpyAsync(dst.rp.p, Hv->rowptr, sizeof(int64_t) * (n + 1), kind, st));
    if (nnz) {
        HIPCHK(hipMemcpyAsync(dst.ci.p, Hv->col, sizeof(int32_t) * nnz, kind, st));
        HIPCHK(hipMemcpyAsync(dst.v.p, Hv->val, sizeof(double) * nnz, kind, st));
    }
    // validate + ||H||_F
    CHK(ensure(P, P.flags, sizeof(int) * 4));
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    HIPCHK(hipMemsetAsync(P.flags.p, 0, sizeof(int), st));
    HIPCHK(validate_csr(dst.view(), nnz, (int *)P.flags.p, st));
    HIPCHK(sumsq((const double *)dst.v.p, nullptr, nnz, (double *)P.part.p, kParts,
                 (double *)P.norm2.p, st));
    HIPCHK(hipMemcpyAsync(P.host, P.flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char *)P.host + 8, P.norm2.p, sizeof(double), hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    int flag;
    double nh2;
    memcpy(&flag, P.host, sizeof flag);
    memcpy(&nh2, (char *)P.host + 8, sizeof nh2);
    if (flag & 1) return fail(EXPM_EINVAL, "rowptr is not a valid CSR row pointer");
    if (flag & 2) return fail(EXPM_EINVAL, "column indices out of range or not strictly increasing");
    if (flag & 4) return fail(EXPM_EINVAL, "H holds NaN or Inf");
    const double nf = sqrt(nh2);
    A->norm_fro = nf;
    A->norm_h = nf;
    if (nf == 0.0) return EXPM_OK;
    if (P.opts.norm == EXPM_NORM_ONE) {
        // the largest column sum: row sums of H^T, each in row order of H
        DCsr Ht;
        auto free_ht = at_exit([&] { release(P, Ht); });
        CHK(transpose_csr(P, dst, Ht));
        CHK(ensure(P, P.amax, sizeof(unsigned long long) * 2));
        HIPCHK(row_abs_max(Ht.view(), (unsigned long long *)P.amax.p, st));
        HIPCHK(hipMemcpyAsync(P.host, P.amax.p, sizeof(double), hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        memcpy(&A->norm_h, P.host, sizeof(double));
    }
    const double nh = A->norm_h;
    int M, N;
    int s = plan_mn(nh, eps, &M, &N);
    if (s == EXPM_ERANGE) return fail(EXPM_ERANGE, "no (M, N) satisfies problem (4.20)");
    if (s) return fail(s, "invalid norm %g", nh);
    if (N >= EXPM_MAXSTEP - 1 || M >= EXPM_MAXSTEP - 1)
        return fail(EXPM_ERANGE, "(M, N) = (%d, %d) exceeds the step limit", M, N);
    int normal = P.opts.normal;
    if (normal < 0) CHK(detect_normal(P, dst, nf, &normal));
    double a = 1.0 / (N + 1);
    if (!normal && (P.opts.literal_a || 1.0 / nh < a)) a = 1.0 / nh;
    if (P.opts.filter_mode != EXPM_FILTER_PAPER) a = 0.0;
    A->M = M;
    A->N = N;
    A->normal = normal;
    A->a = a;
    A->h0 = ldexp(nh, -N);
    A->r0 = plan_r0(M, A->h0);
    A->eg0 = a * A->r0 / (M * exp(2.0 * A->h0));
    return EXPM_OK;
}

int forward(expm_plan_s &P, const expm_csr_cview *Hv, double eps, expm_csr *E) {
    CHK(check_view(Hv));
    if (!E) return fail(EXPM_EINVAL, "E is NULL");
    memset(E, 0, sizeof *E);
    if (!(eps >= ldexp(1.0, -60) && eps < 1.0))
        return fail(EXPM_EINVAL, "eps = %g outside [2^-60, 1)", eps);
    hipStream_t st = P.st;
    const int64_t n = Hv->n, nnz = Hv->nnz;
    free_adjoint_state(P);
    std::fill(P.cts_ok.begin(), P.cts_ok.end(), 0);
    memset(&P.stats, 0, sizeof P.stats);
    // the iterate buffers that rotate through the checkpoints take the size
    // of the last call's T_N (no effect on a first call)
    if (P.opts.keep_checkpoints) {
        CHK(reserve_as(P, P.T, P.TN));
        CHK(reserve_as(P, P.Tnew, P.TN));
        for (DCsr &A : P.ckpt_pool) CHK(reserve_as(P, A, P.TN));
    }
    P.have_stats = false;
    P.perm_active = false;
    P.peak = P.live;
    if (n == 0) {
        E->n = 0;
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, 0, 0, &rp, &ci, &v));
        if (!P.arena) {   // only the row pointer is handed out
            out_free(P, ci);
            out_free(P, v);
        }
        HIPCHK(hipMemsetAsync(rp, 0, sizeof(int64_t), st));
        E->rowptr = rp;
        P.have_stats = true;
        return EXPM_OK;
    }
    TraceRange phase("expm plan (steps 1-3)");
    expm_analysis A{};
    P.last_sym = -1;
    P.sym_h = false;
    CHK(plan_input(P, Hv, eps, P.H0, &A));
    expm_stats &S = P.stats;
    const double nh = A.norm_h;
    S.norm_h = nh;
    if (A.norm_fro == 0.0) {
        P.zero_h = true;
        CHK(output_identity(P, n, E));
        P.Epat.n = 0;
        P.have_fwd = P.opts.keep_checkpoints != 0;
        S.nnz_e = n;
        P.have_stats = true;
        return EXPM_OK;
    }
    P.zero_h = false;
    const int M = A.M, N = A.N;
    const double a = A.a;
    S.M = M;
    S.N = N;
    S.normal = A.normal;
    S.a = a;
    const bool fpim = P.opts.filter_mode == EXPM_FILTER_FIXED_REL;
    P.fpim_eps = fpim ? eps : 0.0;
    // Exactly symmetric H: every T_i is symmetric, so the tile products form
    // only the candidate's upper triangle (T_0, symmetric up to rounding, is
    // made exactly symmetric first)
    if (P.opts.use_symmetry && N >= 1 && tiles_allowed(P, n)) {
        int sym = P.last_sym;
        if (sym < 0) CHK(exact_symmetry(P, P.H0, &sym));
        P.sym_h = sym == 1;
    }
    const bool diag = P.opts.diagnostics != 0;
    for (int i = 0; i < EXPM_MAXSTEP; ++i) S.sq_band[i] = -1;
    if (diag) CHK(ensure(P, P.bands, sizeof(long long) * 2 * (N + 1)));
    const bool keep = P.opts.keep_checkpoints != 0;
    // Locality reordering: H' = P H P^T replaces H; E is permuted back below.
    {
        const int ro = P.opts.reorder;
        P.ordering = 0;
        if (ro >= 1 || (ro < 0 && n >= 4096 && tiles_allowed(P, n)))
            CHK(compute_reorder(P, P.H0.view(), nnz, ro == 2 ? 2 : 1, &P.perm_active));
        S.ordering = P.perm_active ? P.ordering : 0;
        if (P.perm_active) {
            CHK(ensure_csr(P, P.Hp, n, nnz));
            int64_t *hm = nullptr;
            if (keep) {
                CHK(ensure(P, P.hmap, sizeof(int64_t) * (nnz + 1)));
                hm = (int64_t *)P.hmap.p;
            }
            CHK(permute_csr(P, P.H0.view(), nnz, (const int32_t *)P.order.p,
                            (const int32_t *)P.newidx.p, (int64_t *)P.Hp.rp.p,
                            (int32_t *)P.Hp.ci.p, (double *)P.Hp.v.p, hm));
            std::swap(P.H0, P.Hp);
        }
    }
    phase.next("expm taylor seed");
    const auto t_taylor0 = std::chrono::steady_clock::now();
    // Step 3: H0 = H 2^-N, r0, eg0, Taylor seed.
    HIPCHK(scale_ldexp((const double *)P.H0.v.p, (double *)P.H0.v.p, nnz, -N, st));
    const double h0 = A.h0, r0 = A.r0, eg0 = A.eg0;
    S.h0 = h0;
    S.r0 = r0;
    S.eg0 = eg0;
    P.M = M;
    P.N = N;
    P.a = a;
    // Checkpoints of the squaring iterates (the adjoint recomputes the rest):
    // with checkpoint_interval c >= 1, every c-th iterate counted back from
    // T_{N-1}; with -1, ceil(sqrt(N)) of them, on the last iterates
    // T_{N-C} .. T_{N-1}.  Every iterate that is not a checkpoint is
    // recomputed exactly once, and the iterates grow with every squaring,
    // so the last ones are the most expensive to recompute; the early ones
    // the first segment then holds are small.  With 0 (the default) the
    // earlier iterates are kept too, one after another, while their CSR
    // arrays fit in a sixteenth of the device memory: then nothing is
    // recomputed (the checkpoints' tile sets, kept within their own budget,
    // also spare the adjoint the tile assembly).
    const int ci_opt = P.opts.checkpoint_interval;
    const bool ck_last = ci_opt <= 0;
    const bool ck_fill = ci_opt == 0;
    const int ck = ck_last ? std::max(1, (int)ceil(sqrt((double)N))) : ci_opt;
    P.ck = ck;
    size_t extra_ckpt_bytes = 0;
    // the terms are kept (the adjoint needs them, and T_0 is their sum):
    // each is written straight into its slot, where the next product reads it
    P.taylor.reserve(M + 1);
    CHK(copy_csr(P, push_reuse(P.taylor, P.taylor_pool), P.H0));
    S.taylor_terms = 1;
    const CsrView H0v = P.H0.view();
    for (int i = 2; i <= M; ++i) {
        int64_t cand;
        const DCsr &prev = P.taylor.back();
        CHK(spgemm(P, prev.view(), prev.nnz, H0v, 0.0, (double)i, false, &cand));
        FilterCtl h{};
        int64_t kept;
        CHK(filter_and_count(P, n, cand, eg0, nullptr, false, 0.0, false, &h, &kept));
        S.taylor_theta[i] = h.theta;
        S.taylor_iters[i] = h.iter;
        S.taylor_cand[i] = cand;
        S.taylor_kept[i] = kept;
        if (kept == 0) break;   // later terms are exactly zero
        DCsr &slot = push_reuse(P.taylor, P.taylor_pool);
        CHK(write_filtered(P, n, slot, kept, false, false));
        S.taylor_terms = i;
    }
    P.Mp = S.taylor_terms;
    // T_0 = S_1 + ... + S_M' (Eq. 4.14's sum), term after term
    CHK(sum_taylor(P, P.T));
    S.t_taylor_ms = ms_since(t_taylor0);
    phase.next("expm squarings");
    // T's true nnz (the add only bounds it)
    HIPCHK(hipMemcpyAsync(P.host, (int64_t *)P.T.rp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    memcpy(&P.T.nnz, P.host, sizeof(int64_t));
    if (fpim) {
        // the FPIM's filter of T_0: entries at or below eps ||T_0||_1 leave
        // (T_0's buffers serve as the candidate, and the kept entries go
        // back to T_0's buffers)
        auto swap_cand = [&] {
            std::swap(P.crp, P.T.rp);
            std::swap(P.cci, P.T.ci);
            std::swap(P.cv, P.T.v);
        };
        swap_cand();
        CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
        CHK(ensure(P, P.colsum, sizeof(double) * (n + 1)));
        CHK(ensure(P, P.amax, sizeof(unsigned long long) * 2));
        HIPCHK(fpim_theta_rows((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                               (const double *)P.cv.p, n, (double *)P.colsum.p,
                               (unsigned long long *)P.amax.p, eps, (FilterCtl *)P.ctl.p, st));
        FilterCtl h{};
        int64_t kept;
        CHK(filter_and_count(P, n, P.T.nnz, 0.0, nullptr, true, -2.0, false, &h, &kept));
        CHK(write_filtered(P, n, P.T, kept, false, false));
        P.T.nnz = kept;
        S.theta0 = h.theta;
    }
    if (P.sym_h) CHK(symmetrize_upper(P, P.T));
    S.symmetric = P.sym_h ? 1 : 0;
    if (diag) HIPCHK(band_of(P.T.view(), P.perm_active ? (const int32_t *)P.order.p : nullptr,
                            (long long *)P.bands.p, st));
    // The current iterate; a checkpoint takes over P.T's buffers (no copy)
    // and is read by the next squaring in place.
    const DCsr *cur = &P.T;
    if (keep) {
        P.ckpt.reserve(N + 1);
        P.ckpt_at.push_back(0);
        DCsr &slot = push_reuse(P.ckpt, P.ckpt_pool);
        std::swap(slot, P.T);
        cur = &slot;
    }
    const int ck_off = N >= 1 ? (N - 1) % ck : 0;
    auto is_ckpt = [&](int i) {
        return ck_last ? i >= N - ck : i >= ck_off && (i - ck_off) % ck == 0;
    };
    // Step 4: squarings.  Step 5 (E = I + T_N) is fused into the last one.
    DCsr Eout;
    if (keep && (int)P.cts.size() < N + 1) {
        P.cts.resize(N + 1);
        P.cts_ok.resize(N + 1, 0);
    }
    // tile sets of the checkpoints other than T_{N-1} are kept while their
    // total stays within an eighth of the device memory
    if (P.dev_mem == 0) {
        int dev = 0;
        size_t tot = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceTotalMem(&tot, dev) == hipSuccess)
            P.dev_mem = tot;
        (void)hipGetLastError();
    }
    size_t kept_tiles = 0;
    int cur_ck = keep ? 0 : -1;   // checkpoint index of *cur, or -1
    double ri = r0;
    for (int i = 1; i <= N; ++i) {
        // Eq. (4.3): r_i = 2 r_{i-1} + r_{i-1}^2, or its simplification 2^i r0
        ri = P.opts.exact_ri ? 2.0 * ri + ri * ri : ldexp(r0, i);
        S.sq_ri[i] = ri;
        const bool last = i == N;
        CHK(square_step(P, *cur, P.Tnew, a * ri, false, 0.0, false, false, i, i));
        if (diag)
            HIPCHK(band_of(P.Tnew.view(), P.perm_active ? (const int32_t *)P.order.p : nullptr,
                           (long long *)P.bands.p + 2 * i, st));
        if (cur_ck >= 0 && P.sq_path[i - 1]) {   // P.tsT holds the checkpoint's tiles
            const size_t b = P.tsT.tA.bytes + P.tsT.tB.bytes + P.tsT.seg.bytes;
            if (last || kept_tiles + b <= P.dev_mem / 8) {
                std::swap(P.tsT, P.cts[cur_ck]);
                P.cts_ok[cur_ck] = 1;
                kept_tiles += b;
            }
        }
        P.theta.push_back(S.sq_theta[i]);
        std::swap(P.T, P.Tnew);
        P.T.nnz = S.sq_kept[i];
        cur = &P.T;
        cur_ck = -1;
        bool keep_i = keep && !last && is_ckpt(i);
        if (keep && !last && !keep_i && ck_fill) {
            const size_t b = 12 * (size_t)S.sq_kept[i] + 8 * (size_t)(n + 1);
            if (extra_ckpt_bytes + b <= P.dev_mem / 16) {
                keep_i = true;
                extra_ckpt_bytes += b;
            }
        }
        if (keep_i) {
            P.ckpt_at.push_back(i);
            DCsr &slot = push_reuse(P.ckpt, P.ckpt_pool);
            std::swap(slot, P.T);
            cur = &slot;
            cur_ck = (int)P.ckpt.size() - 1;
        }
    }
    S.squarings = N;
    phase.next("expm finish (E = I + T_N)");
    if (N == 0 && cur != &P.T) CHK(copy_csr(P, P.T, *cur));   // T_0 is also T_N
    if (keep) std::swap(P.TN, P.T);   // T_N stays for the adjoint
    // E = I + T_N: T_N's entries as they are, the diagonal 1 + t (inserted as
    // 1 where T_N has none, left out where 1 + t is exactly zero).  With
    // reordering, the permutation back to the caller's order adds the
    // identity on its way (one pass over T'_N instead of two).
    if (P.perm_active) {
        const DCsr &TNs = keep ? P.TN : P.T;
        CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
        int64_t kept = 0, gw = 0;
        CHK(permute_count(P, TNs.view(), (const int32_t *)P.newidx.p, (const int32_t *)P.order.p,
                          (int64_t *)P.krp.p, true, &kept, &gw));
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, n, kept, &rp, &ci, &v));
        HIPCHK(hipMemcpyAsync(rp, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                              st));
        int64_t *tm = nullptr;
        if (keep) {
            CHK(ensure(P, P.tmap, sizeof(int64_t) * (TNs.nnz + 1)));
            tm = (int64_t *)P.tmap.p;
        }
        CHK(permute_write(P, TNs.view(), TNs.nnz, (const int32_t *)P.newidx.p,
                          (const int32_t *)P.order.p, rp, ci, v, nullptr, tm, gw, false, true));
        E->n = n;
        E->nnz = kept;
        E->rowptr = rp;
        E->col = ci;
        E->val = v;
        S.nnz_e = kept;
        if (keep) {   // the adjoint reads dL/dE through tmap, not E's pattern
            P.Epat.n = n;
            P.Epat.nnz = kept;
        }
    } else {
        // T_N becomes the candidate of the compaction (buffers handed over,
        // not copied, and handed back to P.TN after the write when kept)
        DCsr &TNs = keep ? P.TN : P.T;
        auto swap_cand = [&] {
            std::swap(P.crp, TNs.rp);
            std::swap(P.cci, TNs.ci);
            std::swap(P.cv, TNs.v);
        };
        swap_cand();
        FilterCtl h{};
        int64_t kept;
        CHK(filter_and_count(P, n, TNs.nnz, 0.0, nullptr, true, -1.0, true, &h, &kept));
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, n, kept, &rp, &ci, &v));
        HIPCHK(hipMemcpyAsync(rp, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                              st));
        HIPCHK(write_kept((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                          (const double *)P.cv.p, n, (const FilterCtl *)P.ctl.p, 1, rp, ci, v,
                          st));
        if (keep) swap_cand();
        E->n = n;
        E->nnz = kept;
        E->rowptr = rp;
        E->col = ci;
        E->val = v;
        S.nnz_e = kept;
        if (keep) {
            // the adjoint needs E's row pointers (E belongs to the caller):
            // row by row E and T_N differ at most at the diagonal
            CHK(ensure(P, P.Epat.rp, sizeof(int64_t) * (n + 1)));
            HIPCHK(hipMemcpyAsync(P.Epat.rp.p, rp, sizeof(int64_t) * (n + 1),
                                  hipMemcpyDeviceToDevice, st));
            P.Epat.n = n;
            P.Epat.nnz = kept;
        }
    }
    if (diag) {
        long long *hb = (long long *)P.host;
        HIPCHK(hipMemcpyAsync(hb, P.bands.p, sizeof(long long) * 2 * (N + 1),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        for (int i = 0; i <= N; ++i)
            S.sq_band[i] = hb[2 * i] == LLONG_MIN ? 0 : hb[2 * i] + hb[2 * i + 1];
    }
    S.peak_workspace_bytes = P.peak;
    P.have_fwd = keep;
    P.have_stats = true;
    return EXPM_OK;
}

// ------------------------------------------------------------------ backward

// The stored nonzeros of g (values on T's pattern) as a CSR matrix Gc when
// they are fewer than a hundredth of T's entries (*use set), else nothing.
// (At the headline workload a loss on 2% of E's entries still runs faster
// on the tiles of G's whole pattern: 10.8 ms against 12.4 ms for the rows,
// whose transposes of the largest iterate dominate.)
constexpr int64_t kSparseGradDiv = 100;

static int sparse_gradient(expm_plan_s &P, const DCsr &T, const double *g, DCsr &Gc, bool *use) {
    hipStream_t st = P.st;
    const int64_t n = T.n;
    *use = false;
    CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
    FilterCtl *ctl = (FilterCtl *)P.ctl.p;
    HIPCHK(filter_init_theta(ctl, 0.0, st));   // keep |v| > 0
    HIPCHK(count_kept((const int64_t *)T.rp.p, (const int32_t *)T.ci.p, g, n, ctl, 0,
                      (int64_t *)P.cnt.p, st));
    CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.krp.p, n));
    HIPCHK(hipMemcpyAsync(P.host, (int64_t *)P.krp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    int64_t nz;
    memcpy(&nz, P.host, sizeof nz);
    if (nz * kSparseGradDiv >= T.nnz) return EXPM_OK;
    CHK(ensure_csr(P, Gc, n, nz));
    HIPCHK(hipMemcpyAsync(Gc.rp.p, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                          st));
    HIPCHK(write_kept((const int64_t *)T.rp.p, (const int32_t *)T.ci.p, g, n, ctl, 0,
                      (const int64_t *)Gc.rp.p, (int32_t *)Gc.ci.p, (double *)Gc.v.p, st));
    *use = true;
    return EXPM_OK;
}

int backward(expm_plan_s &P, const double *dE, double *dH) {
    if (!P.have_fwd) return fail(EXPM_ESTATE, "no forward state: run expm_sparse with "
                                              "keep_checkpoints = 1 first");
    hipStream_t st = P.st;
    const int64_t n = P.H0.n, nnzH = P.H0.nnz;
    if (P.zero_h) {   // e^0 = I was returned without computation: constant map
        if (nnzH) HIPCHK(hipMemsetAsync(dH, 0, sizeof(double) * nnzH, st));
        return EXPM_OK;
    }
    const int N = P.N;
    // G_N on supp(T_N): E = I + T_N, dL/dT_N = dL/dE at T_N's entries.
    Buf g, gn, dHp, tv, t2v;
    DCsr Tt, H0t, St, Snt, Gc, Gct;
    Buf acc, acc2;
    std::vector<Buf> D;
    auto free_locals = at_exit([&] {
        for (Buf *b : {&g, &gn, &dHp, &acc, &acc2, &tv, &t2v}) release(P, *b);
        for (DCsr *m : {&Tt, &H0t, &St, &Snt, &Gc, &Gct}) release(P, *m);
        for (auto &b : D) release(P, b);
    });
    CHK(ensure(P, g, sizeof(double) * (P.TN.nnz + 1)));
    MaskTerm none{empty_view(), empty_view(), 0.0};
    if (P.perm_active) {
        // each entry of T'_N reads its entry of E through tmap (a diagonal
        // that I + T_N left out reads 0)
        CHK(gather_map(P, dE, (const int64_t *)P.tmap.p, P.TN.nnz, (double *)g.p));
    } else {
        HIPCHK(values_at_t((const int64_t *)P.TN.rp.p, (const int32_t *)P.TN.ci.p,
                           (const int64_t *)P.Epat.rp.p, dE, n, (double *)g.p, st));
    }
    // iterates of the current segment: seg[j] = T^_{base + j} (buffers kept
    // by the plan from call to call)
    std::vector<DCsr> &seg = P.seg_pool;
    int seg_base = -1;
    // The forward kept the tiles of the checkpoint iterates it multiplied
    // (T^_{N-1}'s, the largest, always); the tile sets that trade places
    // below take that size once, so later calls allocate nothing.
    const int lastc = (int)P.ckpt_at.size() - 1;
    const bool fwd_tiles = N >= 1 && lastc >= 0 && lastc < (int)P.cts_ok.size() &&
                           P.cts_ok[lastc] && P.ckpt_at[lastc] == N - 1;
    if (fwd_tiles) {
        const TileSet ref = P.cts[lastc];   // sizes only
        CHK(reserve_as(P, P.tsT, ref));
        CHK(reserve_as(P, P.tsG, ref));
        CHK(reserve_as(P, P.adj_tiles, ref.tB));
        CHK(reserve_as(P, P.adj_tilesA, ref.tA));
    }
    TraceRange phase("expm adjoint squarings");
    const DCsr *Tk = &P.TN;   // pattern of g
    bool g_ready = false;     // P.tsG already holds Tk's tile pattern
    bool g_tiles = false;     // ... and g's values as tiles
    bool g_stale = false;     // g's values only as tiles (P.tsG), not yet in g
    for (int k = N; k >= 1; --k) {
        const int km1 = k - 1;
        // the segment holding T_{k-1}: from the last checkpoint at or below
        // it up to the next checkpoint (or T_N)
        int ci = 0;
        while (ci + 1 < (int)P.ckpt_at.size() && P.ckpt_at[ci + 1] <= km1) ++ci;
        const int base = P.ckpt_at[ci];
        const int next = ci + 1 < (int)P.ckpt_at.size() ? P.ckpt_at[ci + 1] : N;
        const DCsr *Tp;
        if (km1 == base) {
            Tp = &P.ckpt[ci];
        } else {
            if (seg_base != base) {
                if ((int)seg.size() < next - base) seg.resize(next - base);
                seg_base = base;
                const DCsr *prev = &P.ckpt[ci];
                for (int j = base + 1; j <= std::min(next - 1, N - 1); ++j) {
                    CHK(square_step(P, *prev, seg[j - base], 0.0, true, P.theta[j - 1], false,
                                    false, 0, j));
                    prev = &seg[j - base];
                }
            }
            Tp = &seg[km1 - base];
        }
        CHK(ensure(P, gn, sizeof(double) * (Tp->nnz + 1)));
        // The incoming gradient dL/dE is often mostly exact zeros (a loss on
        // a few entries of E).  The first step then runs on the rows of its
        // nonzeros alone: G T^T and T^T G take products only with them, far
        // fewer than the dense tiles of G's whole pattern would.
        bool sparse_g = false;
        if (k == N && Tk->nnz > 0)
            CHK(sparse_gradient(P, *Tk, (const double *)g.p, Gc, &sparse_g));
        // tiles exactly where forward step k ran on tiles (the same test of
        // T_{k-1}'s tile fill)
        const bool tiles = !sparse_g && (int)P.sq_path.size() >= k && P.sq_path[k - 1] != 0;
        bool have_pattern = false, t_ready = false;
        if (tiles) {
            if (km1 == base && ci < (int)P.cts_ok.size() && P.cts_ok[ci]) {
                std::swap(P.tsT, P.cts[ci]);   // kept by the forward
                P.cts_ok[ci] = 0;
                t_ready = true;
            } else {
                double fill = 0.0;
                CHK(bsr_pattern(P, Tp->view(), Tp->nnz, P.tsT, &fill));
            }
            have_pattern = true;
        }
        if (tiles) {
            CHK(adjoint_step_bsr(P, *Tp, *Tk, (const double *)g.p, (double *)gn.p, g_ready,
                                 g_tiles, false, t_ready));
        } else if (sparse_g) {
            // out = P(2 G + G T^T) + P(T^T G), the second term taken as the
            // transpose of P^T(G^T T): every product then pairs a short row
            // (of G or G^T) with long rows of T^T or T.  Tt holds T^T's
            // pattern with the positions of its entries in T, Tv its values.
            CHK(transpose_pos(P, *Tp, Tt));
            CHK(ensure(P, tv, sizeof(double) * (Tp->nnz + 1)));
            CHK(ensure(P, t2v, sizeof(double) * (Tp->nnz + 1)));
            HIPCHK(gather_pos((const double *)Tp->v.p, (const int64_t *)Tt.v.p, Tp->nnz,
                              (double *)tv.p, st));
            const CsrView Ttv{n, (const int64_t *)Tt.rp.p, (const int32_t *)Tt.ci.p,
                              (const double *)tv.p};
            const MaskTerm t1{Gc.view(), Ttv, 1.0};
            CHK(masked(P, Tp->view(), Gc.view(), 2.0, t1, none, 1.0, (double *)gn.p));
            CHK(transpose_csr(P, Gc, Gct));
            const MaskTerm t2{Gct.view(), Tp->view(), 1.0};
            CHK(masked(P, Ttv, empty_view(), 0.0, t2, none, 1.0, (double *)t2v.p));
            HIPCHK(add_scatter_pos((const double *)t2v.p, (const int64_t *)Tt.v.p, Tp->nnz,
                                   (double *)gn.p, st));
            P.stats.adj_sparse_first = 1;
        } else {
            if (g_stale) CHK(gather_tiles(P, *Tk, P.tsG, (const double *)P.tsG.tB.p,
                                          (double *)g.p));
            CHK(transpose_csr(P, *Tp, Tt));
            CsrView Gk = CsrView{n, (const int64_t *)Tk->rp.p, (const int32_t *)Tk->ci.p,
                                 (const double *)g.p};
            MaskTerm t1{Gk, Tt.view(), 1.0}, t2{Tt.view(), Gk, 1.0};
            CHK(masked(P, Tp->view(), Gk, 2.0, t1, t2, 1.0, (double *)gn.p));
        }
        std::swap(g, gn);
        Tk = Tp;
        // T_{k-1}'s tile pattern is the pattern of the next step's gradient:
        // keep it in tsG (recomputation below reuses tsT)
        if (have_pattern) std::swap(P.tsT, P.tsG);
        g_ready = have_pattern;
        // after a tile step the new gradient is already on T_{k-1}'s tiles:
        // its tile buffers become G's, T_{k-1}'s values go to the spare pair
        g_tiles = tiles;
        g_stale = tiles;
        if (tiles) {
            std::swap(P.tsG.tB, P.adj_tiles);
            std::swap(P.tsG.tA, P.adj_tilesA);
        }
        if (k - 1 == base && seg_base == base) seg_base = -1;
    }
    if (g_stale)
        CHK(gather_tiles(P, *Tk, P.tsG, (const double *)P.tsG.tB.p, (double *)g.p));
    // The checkpoints' tile sets trade places with P.tsT in the next forward:
    // they take its size now (they are all free), within the same budget
    // as the kept tiles, so that later calls allocate nothing.
    if (fwd_tiles) {
        const size_t one = P.tsT.tA.bytes + P.tsT.tB.bytes + P.tsT.seg.bytes;
        if ((size_t)P.ckpt_at.size() * one <= P.dev_mem / 8)
            for (size_t c = 0; c < P.ckpt_at.size() && c < P.cts.size(); ++c)
                CHK(reserve_as(P, P.cts[c], P.tsT));
    }
    // Taylor seed: g is dL/dT^_0 on supp(T^_0) = P.ckpt[0].
    phase.next("expm adjoint taylor seed");
    const int Mp = (int)P.taylor.size();
    CsrView G0 = CsrView{n, (const int64_t *)P.ckpt[0].rp.p, (const int32_t *)P.ckpt[0].ci.p,
                         (const double *)g.p};
    CHK(transpose_csr(P, P.H0, H0t));
    D.resize(Mp + 1);
    CHK(ensure(P, D[Mp], sizeof(double) * (P.taylor[Mp - 1].nnz + 1)));
    CHK(masked(P, P.taylor[Mp - 1].view(), G0, 1.0, none, none, 1.0,
               (double *)D[Mp].p));
    CHK(ensure(P, acc, sizeof(double) * (nnzH + 1)));
    CHK(ensure(P, acc2, sizeof(double) * (nnzH + 1)));
    if (nnzH) HIPCHK(hipMemsetAsync(acc.p, 0, sizeof(double) * nnzH, st));
    // acc accumulates sum_i (S^_i^T D_{i+1}) / (i+1) on H's pattern.  Each of
    // its entries is an inner product of a column of S^_i with a column of
    // D_{i+1} (whose pattern is that of S^_{i+1}), so both terms are taken
    // by columns: St and Snt hold the transposed patterns of S^_i and
    // S^_{i+1} with the positions of their entries in the untransposed ones.
    if (Mp >= 2) CHK(transpose_pos(P, P.taylor[Mp - 1], Snt));
    for (int i = Mp - 1; i >= 1; --i) {
        const DCsr &Si = P.taylor[i - 1], &Sn = P.taylor[i];
        CsrView Dn = CsrView{n, (const int64_t *)Sn.rp.p, (const int32_t *)Sn.ci.p,
                             (const double *)D[i + 1].p};
        CHK(ensure(P, D[i], sizeof(double) * (Si.nnz + 1)));
        MaskTerm t1{Dn, H0t.view(), 1.0};
        CHK(masked(P, Si.view(), G0, 1.0, t1, none, (double)(i + 1), (double *)D[i].p));
        CHK(transpose_pos(P, Si, St));
        const PosCsr a{(const int64_t *)St.rp.p, (const int32_t *)St.ci.p,
                       (const int64_t *)St.v.p, (const double *)Si.v.p};
        const PosCsr bt{(const int64_t *)Snt.rp.p, (const int32_t *)Snt.ci.p,
                        (const int64_t *)Snt.v.p, (const double *)D[i + 1].p};
        HIPCHK(masked_dot(P.H0.view(), (const double *)acc.p, a, bt, (double)(i + 1),
                          (double *)acc2.p, st));
        std::swap(acc, acc2);
        std::swap(St, Snt);
    }
    // dH = 2^-N (acc + D_1); S^_1 = H0 shares H's pattern (H' with reordering,
    // whose entries hmap sends back to H's).
    if (P.perm_active) {
        CHK(ensure(P, dHp, sizeof(double) * (nnzH + 1)));
        HIPCHK(add_scaled_ldexp((const double *)acc.p, (const double *)D[1].p,
                                (double *)dHp.p, nnzH, -N, st));
        CHK(scatter_map(P, (const double *)dHp.p, (const int64_t *)P.hmap.p, nnzH, dH));
    } else {
        HIPCHK(add_scaled_ldexp((const double *)acc.p, (const double *)D[1].p, dH, nnzH, -N,
                                st));
    }
    for (auto &b : D) release(P, b);
    release(P, acc);
    release(P, acc2);
    release(P, g);
    release(P, gn);
    release(P, dHp);
    release(P, Tt);
    release(P, H0t);
    release(P, St);
    release(P, Snt);
    CHK(sync(P));
    return EXPM_OK;
}

}  // namespace host
}  // namespace xpm

// ============================================================ fixed region
// The workspace of expm_sparse_noalloc: one static device array per GPU,
// held from the library's load until the process ends.  In host code its
// name is only a host-side handle; the device address of each GPU's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is handed to kernels and copies.
namespace {
static __device__ __align__(256) char scratch[EXPM_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up on first use.
int scratch_address(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EXPM_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(EXPM_EHIP, "no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return EXPM_OK;
}
}  // namespace

// EXPM_LOG=1 in the environment: one line per expm_sparse call on stderr
// with the plan of steps 1-3 and, per squaring, the kept entries, the
// threshold and the filter passes.
void xpm::host::log_call(const expm_plan_s &P, int64_t n, double eps, int status) {
    static const bool on = [] {
        const char *e = getenv("EXPM_LOG");
        return e && atoi(e) > 0;
    }();
    if (!on) return;
    const expm_stats &S = P.stats;
    std::string line;
    char buf[160];
    snprintf(buf, sizeof buf, "expm: n=%lld eps=%.3g status=%d M=%d N=%d normal=%d a=%.4g "
             "||H||=%.6g taylor_terms=%d nnz(E)=%lld", (long long)n, eps, status, S.M, S.N,
             S.normal, S.a, S.norm_h, S.taylor_terms, (long long)S.nnz_e);
    line += buf;
    for (int i = 1; i <= S.squarings && i < EXPM_MAXSTEP; ++i) {
        snprintf(buf, sizeof buf, " | %d: kept=%lld theta=%.3g iters=%d%s", i,
                 (long long)S.sq_kept[i], S.sq_theta[i], S.sq_iters[i],
                 S.sq_tiles[i] ? " tiles" : "");
        line += buf;
    }
    fprintf(stderr, "%s\n", line.c_str());
}

// ====================================================================== C ABI

extern "C" {

void expm_opts_default(expm_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->normal = EXPM_NORMAL_AUTO;
    o->filter_mode = EXPM_FILTER_PAPER;
    o->e_r = 0.1;
    o->max_filter_iter = 64;
    o->keep_checkpoints = 0;
    o->checkpoint_interval = 0;
    o->stream = nullptr;
    o->allocator = nullptr;
    o->reorder = -1;
    o->tile_min_fill = -1.0;
    o->norm = EXPM_NORM_FRO;
    o->exact_ri = 0;
    o->diagnostics = 0;
    o->literal_a = 0;
    o->batch_solo_n = 4096;
    o->use_symmetry = 1;
}

int expm_plan(expm_plan_t *out, const expm_opts *opts) {
    g_err.clear();
    if (!out) return fail(EXPM_EINVAL, "out is NULL");
    *out = nullptr;
    expm_opts o;
    if (opts)
        o = *opts;
    else
        expm_opts_default(&o);
    if (o.filter_mode != EXPM_FILTER_PAPER && o.filter_mode != EXPM_FILTER_NONE &&
        o.filter_mode != EXPM_FILTER_FIXED_REL)
        return fail(EXPM_EINVAL, "unknown filter_mode %d", o.filter_mode);
    if (o.norm != EXPM_NORM_FRO && o.norm != EXPM_NORM_ONE)
        return fail(EXPM_EINVAL, "unknown norm %d", o.norm);
    if (o.exact_ri < 0 || o.exact_ri > 1 || o.diagnostics < 0 || o.diagnostics > 1 ||
        o.literal_a < 0 || o.literal_a > 1 || o.batch_solo_n < 0 || o.use_symmetry < 0 ||
        o.use_symmetry > 1)
        return fail(EXPM_EINVAL, "invalid option value");
    if (!(o.e_r >= 0.0) || o.max_filter_iter < 1 || o.normal < -1 || o.normal > 1 ||
        o.checkpoint_interval < -1 || o.reorder < -1 || o.reorder > 2 || o.profile < 0 ||
        o.profile > 2 ||
        !(o.tile_min_fill == o.tile_min_fill))
        return fail(EXPM_EINVAL, "invalid option value");
    expm_plan_s *P = new (std::nothrow) expm_plan_s();
    if (!P) return fail(EXPM_ENOMEM, "cannot allocate the plan");
    P->opts = o;
    P->st = (hipStream_t)o.stream;
    if (o.tile_min_fill >= 0.0) P->bsr_min_fill = o.tile_min_fill;
    if (hipHostMalloc((void **)&P->host, 4096, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete P;
        return fail(EXPM_EHIP, "cannot allocate pinned host memory");
    }
    // keep freed pool memory cached in the process for reuse between calls
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    }
    (void)hipGetLastError();
    // the shadow plan of expm_sparse_noalloc and the current device's
    // scratch address (set up here, so that the call itself looks up nothing)
    P->na = new (std::nothrow) expm_plan_s();
    void *sp = nullptr;
    const int ss = P->na ? scratch_address(&sp) : fail(EXPM_ENOMEM, "cannot allocate the plan");
    if (ss != EXPM_OK) {
        delete P->na;
        (void)hipHostFree(P->host);
        delete P;
        return ss;
    }
    if (o.profile) {
        P->have_events = true;
        for (hipEvent_t &e : P->ev)
            if (hipEventCreate(&e) != hipSuccess) P->have_events = false;
        (void)hipGetLastError();
    }
    *out = P;
    return EXPM_OK;
}


int expm_sparse(expm_plan_t p, const expm_csr_cview *H, double eps, expm_csr *E) {
    g_err.clear();
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    collect_forward(*p);
    const auto t0 = std::chrono::steady_clock::now();
    p->kt_used = 0;
    p->kt_kind.clear();
    const bool lazy = light_profile(*p);
    if (lazy) (void)hipEventRecord(p->ev[6], p->st);
    int s = forward(*p, H, eps, E);
    if (s == EXPM_OK) {
        if (lazy) {
            // no wait: the timers are read after a later one
            (void)hipEventRecord(p->ev[7], p->st);
            std::swap(p->kt_ev, p->kt_ev_fwd);
            std::swap(p->kt_kind, p->kt_kind_fwd);
            std::swap(p->kt_used, p->kt_used_fwd);
            p->kt_used = 0;
            p->kt_kind.clear();
            p->fwd_pending = true;
        } else if (p->opts.profile == 1) {
            (void)hipStreamSynchronize(p->st);
            p->stats.t_total_ms = ms_since(t0);
            ktimer_collect(*p);
        } else {
            p->stats.t_total_ms = ms_since(t0);   // host time of the call
        }
    }
    log_call(*p, H ? H->n : 0, eps, s);
    if (s != EXPM_OK) {
        p->stats.status = s;
        (void)hipStreamSynchronize(p->st);
        (void)hipGetLastError();
        if (E) {
            out_free(*p, E->rowptr);
            out_free(*p, E->col);
            out_free(*p, E->val);
            memset(E, 0, sizeof *E);
        }
        free_adjoint_state(*p);
    }
    return s;
}

int expm_sparse_noalloc(expm_plan_t p, const expm_csr_cview *H, double eps, int64_t *E_rowptr,
                        int32_t *E_col, double *E_val, int64_t capacity, int64_t *nnz_e) {
    g_err.clear();
    if (nnz_e) *nnz_e = -1;
    if (!p || !p->na) return fail(EXPM_EINVAL, "plan is NULL");
    CHK(check_view(H));
    if (!E_rowptr || capacity < 0 || (capacity > 0 && (!E_col || !E_val)))
        return fail(EXPM_EINVAL, "invalid output buffers");
    // the smallest workspace any input needs: H's pattern and values twice
    // (the copy and its transpose) and eight row arrays
    const double least = 24.0 * (double)H->nnz + 64.0 * (double)(H->n + 1);
    if (least > (double)EXPM_NOALLOC_SCRATCH_BYTES)
        return fail(EXPM_ENOMEM, "H (n = %lld, nnz = %lld) needs more workspace than the "
                    "%zu-byte static scratch of expm_sparse_noalloc holds",
                    (long long)H->n, (long long)H->nnz, (size_t)EXPM_NOALLOC_SCRATCH_BYTES);
    void *base = nullptr;
    CHK(scratch_address(&base));
    // The call runs on the plan's shadow, reset: its buffers are cut from
    // the scratch afresh (nothing of an earlier call is kept there).
    expm_plan_s &S = *p->na;
    S = expm_plan_s();
    S.opts = p->opts;
    S.opts.keep_checkpoints = 0;
    S.opts.profile = 0;
    S.opts.allocator = nullptr;
    S.st = p->st;
    S.host = p->host;
    S.bsr_min_fill = p->bsr_min_fill;
    S.dev_mem = p->dev_mem;
    S.arena = (char *)base;
    S.arena_bytes = EXPM_NOALLOC_SCRATCH_BYTES;
    S.arena_free[0] = EXPM_NOALLOC_SCRATCH_BYTES;
    S.na_rp = E_rowptr;
    S.na_ci = E_col;
    S.na_v = E_val;
    S.na_cap = capacity;
    // the plan's own forward state does not describe this call
    free_adjoint_state(*p);
    expm_csr E{};
    int s = forward(S, H, eps, &E);
    if (nnz_e && S.na_need >= 0) *nnz_e = S.na_need;
    S.stats.status = s;
    p->stats = S.stats;
    p->have_stats = true;
    S.host = nullptr;
    if (s != EXPM_OK) {
        (void)hipStreamSynchronize(p->st);
        (void)hipGetLastError();
    }
    return s;
}

int expm_sparse_backward(expm_plan_t p, const double *dE_vals, double *dH_vals) {
    g_err.clear();
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    if (p->have_fwd && p->H0.nnz && !dH_vals) return fail(EXPM_EINVAL, "dH is NULL");
    if (p->have_fwd && p->Epat.nnz && !dE_vals) return fail(EXPM_EINVAL, "dE is NULL");
    const auto t0 = std::chrono::steady_clock::now();
    p->kt_used = 0;
    p->kt_kind.clear();
    int s = backward(*p, dE_vals, dH_vals);
    if (s == EXPM_OK) {
        p->stats.t_backward_ms = ms_since(t0);
        collect_forward(*p);   // the backward has waited for the device
        ktimer_collect(*p);
    }
    if (s != EXPM_OK) {
        (void)hipStreamSynchronize(p->st);
        (void)hipGetLastError();
    }
    return s;
}


int expm_get_stats(expm_plan_t p, expm_stats *out) {
    if (!p || !out) return fail(EXPM_EINVAL, "NULL argument");
    if (!p->have_stats) return fail(EXPM_ESTATE, "no call has completed on this plan");
    collect_forward(*p);
    *out = p->stats;
    return EXPM_OK;
}

int expm_analyze(expm_plan_t p, const expm_csr_cview *H, double eps, expm_analysis *out) {
    g_err.clear();
    if (!p || !out) return fail(EXPM_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    CHK(check_view(H));
    if (!(eps >= ldexp(1.0, -60) && eps < 1.0))
        return fail(EXPM_EINVAL, "eps = %g outside [2^-60, 1)", eps);
    if (H->n == 0) return EXPM_OK;
    // a scratch copy of H: the plan's own state (the adjoint's) stays intact
    DCsr Hc;
    auto free_hc = at_exit([&] { release(*p, Hc); });
    const int s = plan_input(*p, H, eps, Hc, out);
    if (s != EXPM_OK) {
        (void)hipStreamSynchronize(p->st);
        (void)hipGetLastError();
    }
    return s;
}

// A device view of A: A itself, or (on_host) a copy in the plan's workspace.
static int device_view(expm_plan_s &P, const expm_csr_cview *A, DCsr &copy, CsrView *out) {
    CHK(check_view(A));
    if (!A->on_host) {
        *out = CsrView{A->n, A->rowptr, A->col, A->val};
        return EXPM_OK;
    }
    CHK(ensure_csr(P, copy, A->n, A->nnz));
    HIPCHK(hipMemcpyAsync(copy.rp.p, A->rowptr, sizeof(int64_t) * (A->n + 1),
                          hipMemcpyHostToDevice, P.st));
    if (A->nnz) {
        HIPCHK(hipMemcpyAsync(copy.ci.p, A->col, sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice,
                              P.st));
        HIPCHK(hipMemcpyAsync(copy.v.p, A->val, sizeof(double) * A->nnz, hipMemcpyHostToDevice,
                              P.st));
    }
    *out = copy.view();
    return EXPM_OK;
}

// Y = A X for a block of m columns: on A's 16 x 16 tiles (matrix cores) when
// its stored entries fill at least kSpmmMinFill of its tiles, else from the
// CSR rows.  *ts receives the tiles when they are built (so that repeated
// products reuse them); tiles_ready says they already hold A's.
constexpr double kSpmmMinFill = 0.15;

static int spmm_any(expm_plan_s &P, CsrView Av, int64_t nnz, int64_t m, const double *X,
                    int64_t ldx, double *Y, int64_t ldy, TileSet &ts, int *use_tiles) {
    if (*use_tiles < 0) {
        *use_tiles = 0;
        if (Av.n > 0 && nnz > 0 && m > 0 && tiles_allowed(P, Av.n)) {
            double fill = 0.0;
            CHK(bsr_pattern(P, Av, nnz, ts, &fill));
            if (fill >= kSpmmMinFill && ts.ntiles < INT32_MAX) {
                CHK(bsr_tiles(P, Av, ts));
                *use_tiles = 1;
            }
        }
    }
    if (*use_tiles)
        HIPCHK(spmm_tiles(Av.n, ts.nb, (const int64_t *)ts.tb.p, (const int32_t *)ts.cols.p,
                          (const double *)ts.tA.p, m, X, ldx, Y, ldy, P.st));
    else
        HIPCHK(spmm(Av, m, X, ldx, Y, ldy, P.st));
    return EXPM_OK;
}

int expm_spmm(expm_plan_t p, const expm_csr_cview *A, int64_t m, const double *X, int64_t ldx,
              double *Y, int64_t ldy) {
    g_err.clear();
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    if (m < 0 || ldx < m || ldy < m) return fail(EXPM_EINVAL, "invalid block shape");
    if (m > 0 && A && A->n > 0 && (!X || !Y)) return fail(EXPM_EINVAL, "X or Y is NULL");
    DCsr copy;
    TileSet ts;
    auto free_locals = at_exit([&] {
        release(*p, copy);
        release(*p, ts);
    });
    CsrView Av;
    CHK(device_view(*p, A, copy, &Av));
    int use_tiles = -1;
    return spmm_any(*p, Av, A->nnz, m, X, ldx, Y, ldy, ts, &use_tiles);
}

int expm_propagate(expm_plan_t p, const expm_csr_cview *E, int64_t m, const double *U0,
                   int steps, double *U) {
    g_err.clear();
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    if (m < 0 || steps < 0) return fail(EXPM_EINVAL, "invalid block shape or step count");
    CHK(check_view(E));
    const int64_t n = E->n;
    if (n == 0 || m == 0) return EXPM_OK;
    if (!U0 || !U) return fail(EXPM_EINVAL, "U0 or U is NULL");
    DCsr copy;
    Buf a, b;
    TileSet ts;
    int use_tiles = -1;
    auto free_locals = at_exit([&] {
        release(*p, copy);
        release(*p, a);
        release(*p, b);
        release(*p, ts);
    });
    CsrView Ev;
    CHK(device_view(*p, E, copy, &Ev));
    const size_t bytes = sizeof(double) * (size_t)n * (size_t)m;
    if (steps == 0) {
        if (U != U0) HIPCHK(hipMemcpyAsync(U, U0, bytes, hipMemcpyDeviceToDevice, p->st));
        return EXPM_OK;
    }
    // U_{k+1} = E U_k through two workspace blocks; the last step writes U
    // (U may be U0: U0 is only read by the first step)
    CHK(ensure(*p, a, bytes));
    CHK(ensure(*p, b, bytes));
    const double *src = U0;
    for (int k = 0; k < steps; ++k) {
        double *dst = k == steps - 1 ? (steps == 1 && U == U0 ? (double *)a.p : U)
                                     : (double *)(k % 2 ? b.p : a.p);
        CHK(spmm_any(*p, Ev, E->nnz, m, src, m, dst, m, ts, &use_tiles));
        src = dst;
    }
    if (src != U) HIPCHK(hipMemcpyAsync(U, src, bytes, hipMemcpyDeviceToDevice, p->st));
    return EXPM_OK;
}

int expm_power_norms(expm_plan_t p, const expm_csr_cview *H, int K, double *out) {
    g_err.clear();
    if (!p || (K > 0 && !out)) return fail(EXPM_EINVAL, "NULL argument");
    if (K < 0) return fail(EXPM_EINVAL, "K < 0");
    expm_plan_s &P = *p;
    DCsr copy, cur;
    auto free_locals = at_exit([&] {
        release(P, copy);
        release(P, cur);
    });
    CsrView Hv;
    CHK(device_view(P, H, copy, &Hv));
    const int64_t n = H->n;
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    auto read_norm = [&](const double *v, int64_t m, double *dst) -> int {
        HIPCHK(sumsq(v, nullptr, m, (double *)P.part.p, kParts, (double *)P.norm2.p, P.st));
        HIPCHK(hipMemcpyAsync(P.host, P.norm2.p, sizeof(double), hipMemcpyDeviceToHost, P.st));
        CHK(sync(P));
        double s2;
        memcpy(&s2, P.host, sizeof s2);
        *dst = sqrt(s2);
        return EXPM_OK;
    };
    if (K == 0) return EXPM_OK;
    CHK(read_norm(Hv.v, H->nnz, &out[0]));
    // cur = H^k, k = 1..K (unfiltered products; structural zeros add nothing)
    CsrView Pk = Hv;
    int64_t nnzk = H->nnz;
    for (int k = 2; k <= K; ++k) {
        int64_t cand;
        CHK(spgemm(P, Pk, nnzk, Hv, 0.0, 1.0, false, &cand));
        CHK(ensure_csr(P, cur, n, cand));
        HIPCHK(hipMemcpyAsync(cur.rp.p, P.crp.p, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToDevice, P.st));
        if (cand) {
            HIPCHK(hipMemcpyAsync(cur.ci.p, P.cci.p, sizeof(int32_t) * cand,
                                  hipMemcpyDeviceToDevice, P.st));
            HIPCHK(hipMemcpyAsync(cur.v.p, P.cv.p, sizeof(double) * cand, hipMemcpyDeviceToDevice,
                                  P.st));
        }
        Pk = cur.view();
        nnzk = cand;
        CHK(read_norm((const double *)cur.v.p, cand, &out[k - 1]));
    }
    return EXPM_OK;
}

int expm_alpha_hat(double ri, int i, int N, double norm, const double *hk, int K,
                   int64_t *out) {
    if (!out || !(ri > 0.0) || (hk && K < 3) || (!hk && !(norm >= 0.0)))
        return fail(EXPM_EINVAL, "invalid argument");
    int64_t best = -1;
    const int m1max = hk ? std::min(170, (K - 1) / 2) : 170;
    for (int N1 = 0; N1 <= 60; ++N1) {
        for (int M1 = 1; M1 <= m1max; ++M1) {
            double h = norm;
            if (hk) {   // h_{M1, .} of Eq. (4.9), before its 2^-(N+N1-i) scaling
                h = 0.0;
                for (int k = M1 + 1; k <= 2 * M1 + 1; ++k) h = std::max(h, pow(hk[k - 1], 1.0 / k));
            }
            const double x = ldexp(h, i - N - N1);
            if (ldexp(plan_r0(M1, x), N1) <= ri) {
                const int64_t cost = (int64_t)M1 << N1;
                if (best < 0 || cost < best) best = cost;
                break;
            }
        }
    }
    *out = best;
    return best < 0 ? fail(EXPM_ERANGE, "no (M1, N1) reaches r_i = %g", ri) : EXPM_OK;
}

void expm_csr_release(expm_plan_t p, expm_csr *E) {
    if (!p || !E) return;
    out_free(*p, E->rowptr);
    out_free(*p, E->col);
    out_free(*p, E->val);
    memset(E, 0, sizeof *E);
}

void expm_free(expm_plan_t p) {
    if (!p) return;
    expm_plan_s &P = *p;
    (void)hipStreamSynchronize(P.st);
    free_adjoint_state(P);
    Buf *bufs[] = {&P.lo, &P.words, &P.woff, &P.ub, &P.cnt, &P.crp, &P.bitmaps, &P.lists,
                   &P.counts, &P.scan_tmp, &P.part, &P.ctl, &P.rowsq, &P.norm2, &P.scratch,
                   &P.soff, &P.sbytes, &P.flags, &P.krp, &P.tmp1, &P.tmp2, &P.cci, &P.cv};
    for (Buf *b : bufs) release(P, *b);
    Buf *tbufs[] = {&P.c_lo, &P.c_words, &P.c_woff, &P.c_cnt, &P.c_tb, &P.c_cols, &P.c_tiles,
                    &P.g_cnt, &P.g_ofs, &P.b_sq, &P.b_nz, &P.tc_cnt, &P.tc_ptr,
                    &P.tc_fill, &P.tc_k, &P.tc_t, &P.adj_tiles, &P.adj_tilesA, &P.c_rt, &P.p_lo,
                    &P.p_words, &P.p_woff, &P.p_cnt, &P.p_ofs, &P.p_gcnt, &P.p_gofs,
                    &P.p_owner, &P.g_owner, &P.p_cols, &P.c_sq, &P.c_nz, &P.c_mn, &P.c_mx, &P.c_rc, &P.c_kc, &P.b_dg};
    for (Buf *b : tbufs) release(P, *b);
    Buf *rbufs[] = {&P.order, &P.newidx, &P.hmap, &P.tmap, &P.ro_rb, &P.ro_d0, &P.ro_d1,
                    &P.ro_d3, &P.ro_q0, &P.ro_q1, &P.ro_ell, &P.ro_cell, &P.ro_cnt, &P.ro_off,
                    &P.ro_pcnt, &P.ro_pw, &P.ro_pofs, &P.ro_gbits};
    for (Buf *b : rbufs) release(P, *b);
    for (Buf *b : {&P.colsum, &P.amax, &P.bands}) release(P, *b);
    for (Buf *b : {&P.mirror_bad, &P.sym_cnt, &P.c_mir, &P.r_cnt, &P.r_ofs, &P.r_rows, &P.r_owner})
        release(P, *b);
    release(P, P.tsT);
    release(P, P.tsG);
    for (TileSet &ts : P.cts) release(P, ts);
    DCsr *mats[] = {&P.H0, &P.S,  &P.Snew, &P.T,     &P.Tnew,
                    &P.Hpat_t, &P.Hp, &P.Eperm, &P.TN, &P.Epat};
    for (DCsr *m : mats) release(P, *m);
    for (auto *v : {&P.taylor_pool, &P.ckpt_pool, &P.seg_pool})
        for (DCsr &A : *v) release(P, A);
    while (!P.outputs.empty()) out_free(P, P.outputs.back());
    (void)hipStreamSynchronize(P.st);
    if (P.have_events)
        for (hipEvent_t &e : P.ev) (void)hipEventDestroy(e);
    for (hipEvent_t &e : P.kt_ev) (void)hipEventDestroy(e);
    for (hipEvent_t &e : P.kt_ev_fwd) (void)hipEventDestroy(e);
    delete P.na;   // its buffers lie in the static scratch: nothing to free
    if (P.host) (void)hipHostFree(P.host);
    (void)hipGetLastError();
    delete p;
}

const char *expm_last_error(void) { return g_err.c_str(); }

double expm_r0(int M, double x) { return plan_r0(M, x); }

int expm_choose_mn(double norm_h, double eps, int *M, int *N) {
    if (!M || !N) return fail(EXPM_EINVAL, "NULL output");
    int s = plan_mn(norm_h, eps, M, N);
    if (s) return fail(s, "no (M, N) for norm %g and eps %g", norm_h, eps);
    return EXPM_OK;
}

}  // extern "C"
