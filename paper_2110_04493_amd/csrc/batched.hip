// Batched exponentials (expm_sparse_batched): many independent matrices in
// one pass of Algorithm 4.2.
//
// The instances are sorted by their squaring count N (largest first) and
// stacked into one block-diagonal CSR, so the product kernels, the bins and
// the row lists serve the rows of every instance in the same launches.  Each
// instance keeps its own scalars (M, N, a, r0 and the budgets of Algorithm
// 4.2) and its own Algorithm 4.1 controller; every row reads the threshold
// of its instance.  Because of the ordering, the instances still squaring at
// step s are a prefix of the stack: step s runs on that prefix of rows and
// the instances that finish at s are cut off the tail with E = I + T_N
// applied in the same compaction.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "plan.hpp"

namespace xpm {

constexpr int kBlk = 256;

__device__ double blk_sum(double s) {
    __shared__ double ws[kBlk / kWave];
    s = wave_sum(s);
    if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int j = 0; j < kBlk / kWave; j++) t += ws[j];
    __syncthreads();
    return t;
}

__global__ void k_fill_row_inst(const int64_t *row_off, int count, int64_t n, int32_t *row_inst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = count - 1;   // last k with row_off[k] <= i
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (row_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    row_inst[i] = lo;
}

hipError_t fill_row_inst(const int64_t *row_off, int count, int64_t n, int32_t *row_inst,
                         hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_row_inst, dim3((n + 255) / 256), dim3(256), 0, st, row_off, count,
                       n, row_inst);
    return hipGetLastError();
}

__global__ void k_filter_init_batched(FilterCtl *c, int count, const double *eg_scale,
                                      const double *norm2, const int *mode, double er, int maxit) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    FilterCtl &f = c[k];
    f.er = er;
    f.maxit = maxit;
    f.iter = 0;
    f.status = 0;
    f.m = 1.0;
    f.arrive = 0;
    f.b = 0.0;
    const int md = mode[k];
    if (md == 1) {            // keep everything (instance not filtered at this step)
        f.eg = 0.0;
        f.theta = -1.0;
        f.done = 1;
        return;
    }
    if (md == 2) {            // drop everything (instance finished its Taylor terms)
        f.eg = 0.0;
        f.theta = INFINITY;
        f.done = 1;
        return;
    }
    const double eg = norm2 ? eg_scale[k] * sqrt(norm2[k]) : eg_scale[k];
    f.eg = eg;
    if (eg > 0.0) {
        f.theta = eg;         // eps_f^(1) = eps_g / m_0
        f.b = INFINITY;
        f.done = 0;
    } else {
        f.theta = 0.0;        // a = 0: only exact zeros leave
        f.done = 1;
    }
}

hipError_t filter_init_batched(FilterCtl *c, int count, const double *eg_scale,
                               const double *norm2, const int *mode, double er, int maxit,
                               hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_init_batched, dim3((count + 255) / 256), dim3(256), 0, st, c,
                       count, eg_scale, norm2, mode, er, maxit);
    return hipGetLastError();
}

// Algorithm 4.1 pass per instance: blocks [k*B, (k+1)*B) sum v^2 over the
// entries of instance k with |v| <= theta_k; the last of them to finish sums
// the B partials in order and advances controller k.
__global__ __launch_bounds__(kBlk) void k_filter_pass_batched(const double *__restrict__ cv,
                                                              const int64_t *crp,
                                                              const int64_t *row_off,
                                                              FilterCtl *ctl, double *part,
                                                              int B) {
    const int k = blockIdx.x / B, b = blockIdx.x % B;
    FilterCtl *c = &ctl[k];
    if (c->done) return;
    const double theta = c->theta;
    const int64_t s = crp[row_off[k]], e = crp[row_off[k + 1]];
    double acc = 0.0;
    for (int64_t j = s + (int64_t)b * kBlk + threadIdx.x; j < e; j += (int64_t)B * kBlk) {
        const double x = cv[j];
        if (fabs(x) <= theta) acc = fma(x, x, acc);
    }
    acc = blk_sum(acc);
    __shared__ unsigned ticket;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        __threadfence();
        ticket = atomicAdd(&c->arrive, 1u);
    }
    __syncthreads();
    if (ticket != (unsigned)B - 1) return;
    __threadfence();
    double t = 0.0;
    for (int j = threadIdx.x; j < B; j += kBlk) t += __builtin_nontemporal_load(&part[k * B + j]);
    t = blk_sum(t);
    if (threadIdx.x == 0) {
        const double bn = sqrt(t);
        c->b = bn;
        c->iter += 1;
        c->arrive = 0;
        if (bn <= c->eg * (1.0 + c->er)) {
            c->done = 1;
        } else if (c->iter >= c->maxit) {
            c->done = 1;
            c->status = 1;
        } else {
            c->m = bn / theta;
            c->theta = c->eg / c->m;
        }
    }
}

hipError_t filter_pass_batched(const double *cv, const int64_t *crp, const int64_t *row_off,
                               int count, FilterCtl *c, double *part, int blocks_per_inst,
                               hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_pass_batched, dim3(count * blocks_per_inst), dim3(kBlk), 0, st,
                       cv, crp, row_off, c, part, blocks_per_inst);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlk) void k_segment_sums(const double *v, const int64_t *row_off,
                                                       double *out) {
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t i = row_off[k] + threadIdx.x; i < row_off[k + 1]; i += kBlk) s += v[i];
    s = blk_sum(s);
    if (threadIdx.x == 0) out[k] = s;
}

hipError_t segment_sums(const double *v, const int64_t *row_off, int count, double *out,
                        hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_segment_sums, dim3(count), dim3(kBlk), 0, st, v, row_off, out);
    return hipGetLastError();
}

__global__ void k_gather_offsets(const int64_t *rp, const int64_t *row_off, int count,
                                 int64_t *out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= count) out[k] = rp[row_off[k]];
}

hipError_t gather_offsets(const int64_t *rp, const int64_t *row_off, int count, int64_t *out,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_gather_offsets, dim3((count + 256) / 256), dim3(256), 0, st, rp, row_off,
                       count, out);
    return hipGetLastError();
}

// One wave per stacked row: copies the instance row with columns shifted to
// the instance's diagonal block and values scaled by 2^-shift.
__global__ void k_stack(const InstDesc *desc, int count, const int64_t *row_off, int64_t n,
                        int64_t *rp, int32_t *ci, double *v) {
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (row_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const InstDesc d = desc[lo];
    const int64_t r = i - d.row_off;
    const int64_t b = d.rp[r], e = d.rp[r + 1], base = d.rp[0];
    const int64_t o = d.nnz_off + (b - base);
    if (lane_id() == 0) {
        rp[i] = o;
        if (i == n - 1) rp[n] = d.nnz_off + (e - base);
    }
    for (int64_t p = b + lane_id(); p < e; p += kWave) {
        ci[o + (p - b)] = d.ci[p] + (int32_t)d.row_off;
        v[o + (p - b)] = ldexp(d.v[p], -d.shift);
    }
}

hipError_t stack_instances(const InstDesc *desc, int count, const int64_t *row_off, int64_t n,
                           int64_t *rp, int32_t *ci, double *v, hipStream_t st) {
    if (n == 0) return hipMemsetAsync(rp, 0, sizeof(int64_t), st);
    int wpb = 4;
    hipLaunchKernelGGL(k_stack, dim3((n + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, desc, count,
                       row_off, n, rp, ci, v);
    return hipGetLastError();
}

__global__ void k_extract(const int64_t *rp, const int32_t *ci, const double *v, int64_t r0,
                          int64_t m, int64_t *orp, int32_t *oci, double *ov) {
    int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= m) return;
    const int64_t base = rp[r0], b = rp[r0 + r], e = rp[r0 + r + 1];
    if (lane_id() == 0) {
        orp[r] = b - base;
        if (r == m - 1) orp[m] = e - base;
    }
    for (int64_t p = b + lane_id(); p < e; p += kWave) {
        oci[p - base] = ci[p] - (int32_t)r0;
        ov[p - base] = v[p];
    }
}

hipError_t extract_block(const int64_t *rp, const int32_t *ci, const double *v, int64_t r0,
                         int64_t m, int64_t *orp, int32_t *oci, double *ov, hipStream_t st) {
    if (m == 0) return hipMemsetAsync(orp, 0, sizeof(int64_t), st);
    int wpb = 4;
    hipLaunchKernelGGL(k_extract, dim3((m + wpb - 1) / wpb), dim3(wpb * kWave), 0, st, rp, ci, v,
                       r0, m, orp, oci, ov);
    return hipGetLastError();
}

// ====================================================================== host

namespace host {
namespace {

struct Inst {
    int idx = 0;          // position in the caller's arrays
    int64_t n = 0, nnz = 0;
    double eps = 0, nh = 0, a = 0, r0 = 0, eg0 = 0;
    int M = 0, N = 0, normal = 0, taylor_done = 0, terms = 1;
    bool zero = false;
};

struct BatchBufs {
    Buf rowoff, rowinst, desc, ctl, egs, modes, addi, norm2, segoff, part;
};

void free_bufs(expm_plan_s &P, BatchBufs &B) {
    Buf *all[] = {&B.rowoff, &B.rowinst, &B.desc, &B.ctl, &B.egs, &B.modes, &B.addi, &B.norm2,
                  &B.segoff, &B.part};
    for (Buf *b : all) release(P, *b);
}

constexpr int kBlocksPerInst = 32;

// Algorithm 4.1 for every instance (controllers initialised by the caller)
// followed by the kept counts of the rows [0, n).
int batched_filter(expm_plan_s &P, BatchBufs &B, int count, int64_t n, const int *inst_addI,
                   std::vector<FilterCtl> &hctl) {
    hipStream_t st = P.st;
    FilterCtl *ctl = (FilterCtl *)B.ctl.p;
    CHK(ensure(P, B.part, sizeof(double) * (size_t)count * kBlocksPerInst));
    CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    hctl.resize(count);
    for (int round = 0;; ++round) {
        for (int j = 0; j < 4; ++j)
            HIPCHK(filter_pass_batched((const double *)P.cv.p, (const int64_t *)P.crp.p,
                                       (const int64_t *)B.rowoff.p, count, ctl,
                                       (double *)B.part.p, kBlocksPerInst, st));
        HIPCHK(hipMemcpyAsync(hctl.data(), ctl, sizeof(FilterCtl) * count, hipMemcpyDeviceToHost,
                              st));
        CHK(sync(P));
        bool all = true;
        for (int k = 0; k < count; ++k) all = all && hctl[k].done;
        if (all) break;
        if (round > P.opts.max_filter_iter)
            return fail(EXPM_ENOTCONV, "Algorithm 4.1 did not stop");
    }
    for (int k = 0; k < count; ++k)
        if (hctl[k].status)
            return fail(EXPM_ENOTCONV, "Algorithm 4.1 reached %d iterations in instance %d",
                        hctl[k].iter, k);
    HIPCHK(count_kept((const int64_t *)P.crp.p, (const int32_t *)P.cci.p, (const double *)P.cv.p,
                      n, ctl, 0, (int64_t *)P.cnt.p, st, (const int32_t *)B.rowinst.p,
                      inst_addI));
    CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.krp.p, n));
    return EXPM_OK;
}

int batched(expm_plan_s &P, BatchBufs &B, int count, const expm_csr_cview *H, const double *eps,
            expm_csr *E) {
    hipStream_t st = P.st;
    if (count < 0) return fail(EXPM_EINVAL, "count < 0");
    if (count > 0 && (!H || !eps || !E)) return fail(EXPM_EINVAL, "NULL array");
    for (int k = 0; k < count; ++k) memset(&E[k], 0, sizeof E[k]);
    free_adjoint_state(P);
    memset(&P.stats, 0, sizeof P.stats);
    P.sym_h = false;   // the stacked products form every candidate tile
    if (count == 0) return EXPM_OK;
    if (P.opts.filter_mode == EXPM_FILTER_FIXED_REL || P.opts.norm != EXPM_NORM_FRO ||
        P.opts.exact_ri)
        return fail(EXPM_ENOTIMPL, "the batched path runs the default filter, norm and error "
                                   "recurrence only");
    for (int k = 0; k < count; ++k)
        if (H[k].on_host) return fail(EXPM_EINVAL, "instance %d: the batched path takes device "
                                                   "views only", k);
    std::vector<Inst> in(count);
    for (int k = 0; k < count; ++k) {
        CHK(check_view(&H[k]));
        if (!(eps[k] >= ldexp(1.0, -60) && eps[k] < 1.0))
            return fail(EXPM_EINVAL, "eps[%d] = %g outside [2^-60, 1)", k, eps[k]);
        in[k].idx = k;
        in[k].n = H[k].n;
        in[k].nnz = H[k].nnz;
        in[k].eps = eps[k];
    }
    // --- validation and ||H_k||_F, per instance
    CHK(ensure(P, P.flags, sizeof(int) * (size_t)count));
    CHK(ensure(P, P.norm2, sizeof(double) * (size_t)count));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    HIPCHK(hipMemsetAsync(P.flags.p, 0, sizeof(int) * count, st));
    for (int k = 0; k < count; ++k) {
        CsrView v{H[k].n, H[k].rowptr, H[k].col, H[k].val};
        if (H[k].n > 0) HIPCHK(validate_csr(v, H[k].nnz, (int *)P.flags.p + k, st));
        HIPCHK(sumsq(H[k].val, nullptr, H[k].nnz, (double *)P.part.p, 64,
                     (double *)P.norm2.p + k, st));
    }
    std::vector<int> hflag(count);
    std::vector<double> hn2(count);
    HIPCHK(hipMemcpyAsync(hflag.data(), P.flags.p, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hn2.data(), P.norm2.p, sizeof(double) * count, hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    for (int k = 0; k < count; ++k) {
        if (hflag[k]) return fail(EXPM_EINVAL, "instance %d is not a valid CSR matrix", k);
        Inst &I = in[k];
        I.nh = sqrt(hn2[k]);
        I.zero = I.nh == 0.0 || I.n == 0;
        if (I.zero) continue;
        int s = plan_mn(I.nh, I.eps, &I.M, &I.N);
        if (s) return fail(s == EXPM_ERANGE ? EXPM_ERANGE : s, "no (M, N) for instance %d", k);
        if (I.M >= EXPM_MAXSTEP - 1 || I.N >= EXPM_MAXSTEP - 1)
            return fail(EXPM_ERANGE, "(M, N) of instance %d exceeds the step limit", k);
    }
    // --- order: largest N first (stable); zero instances last
    std::vector<int> ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        if (in[x].zero != in[y].zero) return !in[x].zero;
        return in[x].N > in[y].N;
    });
    std::vector<Inst> A;   // active (non-zero) instances in stack order
    for (int k : ord)
        if (!in[k].zero) A.push_back(in[k]);
    const int K = (int)A.size();
    std::vector<int64_t> roff(K + 1, 0), noff(K + 1, 0);
    for (int k = 0; k < K; ++k) {
        roff[k + 1] = roff[k] + A[k].n;
        noff[k + 1] = noff[k] + A[k].nnz;
    }
    const int64_t n = roff[K], nnz = noff[K];
    if (n > INT32_MAX - 1) return fail(EXPM_EINVAL, "stacked order %lld too large", (long long)n);
    // zero matrices: E = I
    for (int k = 0; k < count; ++k) {
        if (!in[k].zero) continue;
        const int64_t nk = in[k].n;
        int64_t *rp = (int64_t *)out_alloc(P, sizeof(int64_t) * (nk + 1));
        int32_t *ci = (int32_t *)out_alloc(P, sizeof(int32_t) * nk);
        double *v = (double *)out_alloc(P, sizeof(double) * nk);
        if (!rp || !ci || !v) return fail(EXPM_ENOMEM, "cannot allocate output %d", k);
        HIPCHK(fill_identity(nk, rp, ci, v, st));
        E[k] = expm_csr{nk, nk, rp, ci, v};
    }
    if (K == 0) return EXPM_OK;
    // --- stack H0 = blockdiag(H_k 2^-N_k)
    std::vector<InstDesc> hd(K);
    for (int k = 0; k < K; ++k) {
        const expm_csr_cview &h = H[A[k].idx];
        hd[k] = InstDesc{h.rowptr, h.col, h.val, h.n, roff[k], noff[k], A[k].N};
    }
    CHK(ensure(P, B.rowoff, sizeof(int64_t) * (K + 1)));
    CHK(ensure(P, B.rowinst, sizeof(int32_t) * n));
    CHK(ensure(P, B.desc, sizeof(InstDesc) * K));
    CHK(ensure(P, B.ctl, sizeof(FilterCtl) * K));
    CHK(ensure(P, B.egs, sizeof(double) * K));
    CHK(ensure(P, B.modes, sizeof(int) * K));
    CHK(ensure(P, B.addi, sizeof(int) * K));
    CHK(ensure(P, B.norm2, sizeof(double) * K));
    CHK(ensure(P, B.segoff, sizeof(int64_t) * (K + 1)));
    HIPCHK(hipMemcpyAsync(B.rowoff.p, roff.data(), sizeof(int64_t) * (K + 1),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B.desc.p, hd.data(), sizeof(InstDesc) * K, hipMemcpyHostToDevice, st));
    HIPCHK(fill_row_inst((const int64_t *)B.rowoff.p, K, n, (int32_t *)B.rowinst.p, st));
    CHK(ensure_csr(P, P.H0, n, nnz));
    HIPCHK(stack_instances((const InstDesc *)B.desc.p, K, (const int64_t *)B.rowoff.p, n,
                           (int64_t *)P.H0.rp.p, (int32_t *)P.H0.ci.p, (double *)P.H0.v.p, st));
    // normality: exact symmetry per instance on the stack, commutator test
    // on the instance itself otherwise (Algorithm 4.2 step 2)
    {
        DCsr Ht;
        CHK(transpose_csr(P, P.H0, Ht));
        std::vector<int> nf(K, -1);
        for (int k = 0; k < K; ++k)
            if (P.opts.normal >= 0) nf[k] = P.opts.normal;
        if (P.opts.normal < 0) {
            // compare entry by entry (scaling by 2^-N keeps (skew-)symmetry exact)
            CHK(ensure(P, P.flags, sizeof(int) * 3 * (size_t)K));
            std::vector<int> ones(3 * K, 1);
            HIPCHK(hipMemcpyAsync(P.flags.p, ones.data(), sizeof(int) * 3 * K,
                                  hipMemcpyHostToDevice, st));
            std::vector<int> hf(3 * K);
            for (int k = 0; k < K; ++k) {
                // The transpose of a block-diagonal stack is the stack of the
                // transposes, with the same block boundaries, so the slices
                // of instance k (rows from roff[k], entries from noff[k])
                // compare directly; row pointers stay absolute in both.
                const int64_t nk = A[k].n, e0 = noff[k];
                CsrView a{nk, (const int64_t *)P.H0.rp.p + roff[k],
                          (const int32_t *)P.H0.ci.p + e0, (const double *)P.H0.v.p + e0};
                CsrView b{nk, (const int64_t *)Ht.rp.p + roff[k], (const int32_t *)Ht.ci.p + e0,
                          (const double *)Ht.v.p + e0};
                HIPCHK(compare_csr(a, b, A[k].nnz, (int *)P.flags.p + 3 * k, st));
            }
            HIPCHK(hipMemcpyAsync(hf.data(), P.flags.p, sizeof(int) * 3 * K,
                                  hipMemcpyDeviceToHost, st));
            CHK(sync(P));
            for (int k = 0; k < K; ++k)
                if (hf[3 * k] && (hf[3 * k + 1] || hf[3 * k + 2])) nf[k] = 1;
            for (int k = 0; k < K; ++k) {
                if (nf[k] >= 0) continue;
                const expm_csr_cview &h = H[A[k].idx];
                DCsr Hk;
                CHK(ensure_csr(P, Hk, h.n, h.nnz));
                HIPCHK(hipMemcpyAsync(Hk.rp.p, h.rowptr, sizeof(int64_t) * (h.n + 1),
                                      hipMemcpyDeviceToDevice, st));
                if (h.nnz) {
                    HIPCHK(hipMemcpyAsync(Hk.ci.p, h.col, sizeof(int32_t) * h.nnz,
                                          hipMemcpyDeviceToDevice, st));
                    HIPCHK(hipMemcpyAsync(Hk.v.p, h.val, sizeof(double) * h.nnz,
                                          hipMemcpyDeviceToDevice, st));
                }
                int nm = 0;
                CHK(detect_normal(P, Hk, A[k].nh, &nm));
                nf[k] = nm;
                release(P, Hk);
            }
        }
        release(P, Ht);
        for (int k = 0; k < K; ++k) {
            Inst &I = A[k];
            I.normal = nf[k];
            I.a = 1.0 / (I.N + 1);
            if (!I.normal && (P.opts.literal_a || 1.0 / I.nh < I.a)) I.a = 1.0 / I.nh;
            if (P.opts.filter_mode == EXPM_FILTER_NONE) I.a = 0.0;
            const double h0 = ldexp(I.nh, -I.N);
            I.r0 = plan_r0(I.M, h0);
            I.eg0 = I.a * I.r0 / (I.M * exp(2.0 * h0));
        }
    }
    // --- Taylor seed for all instances at once
    CHK(copy_csr(P, P.S, P.H0));
    CHK(copy_csr(P, push_reuse(P.taylor, P.taylor_pool), P.H0));   // the terms, summed below
    int maxM = 0;
    for (auto &I : A) maxM = std::max(maxM, I.M);
    std::vector<double> egs(K);
    std::vector<int> modes(K), addi(K);
    std::vector<FilterCtl> hctl;
    std::vector<int64_t> seg(K + 1);
    const CsrView H0v = P.H0.view();
    for (int i = 2; i <= maxM; ++i) {
        bool any = false;
        for (int k = 0; k < K; ++k) {
            const bool act = !A[k].taylor_done && i <= A[k].M;
            if (!act) A[k].taylor_done = 1;
            modes[k] = act ? 0 : 2;
            egs[k] = A[k].eg0;
            any = any || act;
        }
        if (!any) break;
        int64_t cand;
        CHK(spgemm(P, P.S.view(), P.S.nnz, H0v, 0.0, (double)i, false, &cand));
        HIPCHK(hipMemcpyAsync(B.egs.p, egs.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(B.modes.p, modes.data(), sizeof(int) * K, hipMemcpyHostToDevice,
                              st));
        HIPCHK(filter_init_batched((FilterCtl *)B.ctl.p, K, (const double *)B.egs.p, nullptr,
                                   (const int *)B.modes.p, P.opts.e_r, P.opts.max_filter_iter,
                                   st));
        CHK(batched_filter(P, B, K, n, nullptr, hctl));
        HIPCHK(gather_offsets((const int64_t *)P.krp.p, (const int64_t *)B.rowoff.p, K,
                              (int64_t *)B.segoff.p, st));
        HIPCHK(hipMemcpyAsync(seg.data(), B.segoff.p, sizeof(int64_t) * (K + 1),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        const int64_t kept = seg[K];
        CHK(ensure_csr(P, P.Snew, n, kept));
        HIPCHK(hipMemcpyAsync(P.Snew.rp.p, P.krp.p, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToDevice, st));
        HIPCHK(write_kept((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                          (const double *)P.cv.p, n, (const FilterCtl *)B.ctl.p, 0,
                          (const int64_t *)P.Snew.rp.p, (int32_t *)P.Snew.ci.p,
                          (double *)P.Snew.v.p, st, (const int32_t *)B.rowinst.p, nullptr));
        std::swap(P.S, P.Snew);
        P.S.nnz = kept;
        for (int k = 0; k < K; ++k) {
            if (modes[k] != 0) continue;
            if (seg[k + 1] == seg[k])
                A[k].taylor_done = 1;   // this term and all later ones are zero
            else
                A[k].terms = i;
        }
        CHK(copy_csr(P, push_reuse(P.taylor, P.taylor_pool), P.S));
    }
    CHK(sum_taylor(P, P.T));
    HIPCHK(hipMemcpyAsync(P.host, (int64_t *)P.T.rp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    memcpy(&P.T.nnz, P.host, sizeof(int64_t));
    // --- squarings on the shrinking prefix of still-active instances
    int maxN = 0;
    for (auto &I : A) maxN = std::max(maxN, I.N);
    int Ka = K;   // active instances = stack prefix [0, Ka)
    auto finish = [&](int s) -> int {
        // instances with N == s are finished after step s (or after the
        // Taylor seed when s == 0): their rows are the tail of the prefix
        int Kn = Ka;
        while (Kn > 0 && A[Kn - 1].N == s) --Kn;
        if (Kn == Ka) return EXPM_OK;
        const int64_t R = roff[Ka];
        if (s == 0) {
            // E = I + T_0 for the N = 0 instances: keep-all compaction
            for (int k = 0; k < Ka; ++k) {
                modes[k] = 1;
                addi[k] = k >= Kn;
            }
            CHK(ensure(P, P.crp, sizeof(int64_t) * (R + 1)));
            CHK(ensure(P, P.cci, sizeof(int32_t) * (P.T.nnz + 1)));
            CHK(ensure(P, P.cv, sizeof(double) * (P.T.nnz + 1)));
            HIPCHK(hipMemcpyAsync(P.crp.p, P.T.rp.p, sizeof(int64_t) * (R + 1),
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(P.cci.p, P.T.ci.p, sizeof(int32_t) * P.T.nnz,
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(P.cv.p, P.T.v.p, sizeof(double) * P.T.nnz,
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(B.modes.p, modes.data(), sizeof(int) * Ka,
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(B.addi.p, addi.data(), sizeof(int) * Ka, hipMemcpyHostToDevice,
                                  st));
            HIPCHK(filter_init_batched((FilterCtl *)B.ctl.p, Ka, (const double *)B.egs.p,
                                       nullptr, (const int *)B.modes.p, P.opts.e_r,
                                       P.opts.max_filter_iter, st));
            CHK(batched_filter(P, B, Ka, R, (const int *)B.addi.p, hctl));
            HIPCHK(gather_offsets((const int64_t *)P.krp.p, (const int64_t *)B.rowoff.p, Ka,
                                  (int64_t *)B.segoff.p, st));
            HIPCHK(hipMemcpyAsync(seg.data(), B.segoff.p, sizeof(int64_t) * (Ka + 1),
                                  hipMemcpyDeviceToHost, st));
            CHK(sync(P));
            CHK(ensure_csr(P, P.Tnew, R, seg[Ka]));
            HIPCHK(hipMemcpyAsync(P.Tnew.rp.p, P.krp.p, sizeof(int64_t) * (R + 1),
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(write_kept((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                              (const double *)P.cv.p, R, (const FilterCtl *)B.ctl.p, 0,
                              (const int64_t *)P.Tnew.rp.p, (int32_t *)P.Tnew.ci.p,
                              (double *)P.Tnew.v.p, st, (const int32_t *)B.rowinst.p,
                              (const int *)B.addi.p));
        }
        // P.Tnew holds the compacted rows [0, R) (with I added for the
        // finished tail); copy each finished instance out
        for (int k = Kn; k < Ka; ++k) {
            const int64_t nk = A[k].n, ek = seg[k + 1] - seg[k];
            int64_t *rp = (int64_t *)out_alloc(P, sizeof(int64_t) * (nk + 1));
            int32_t *ci = (int32_t *)out_alloc(P, sizeof(int32_t) * ek);
            double *v = (double *)out_alloc(P, sizeof(double) * ek);
            if (!rp || !ci || !v) return fail(EXPM_ENOMEM, "cannot allocate output");
            HIPCHK(extract_block((const int64_t *)P.Tnew.rp.p, (const int32_t *)P.Tnew.ci.p,
                                 (const double *)P.Tnew.v.p, roff[k], nk, rp, ci, v, st));
            E[A[k].idx] = expm_csr{nk, ek, rp, ci, v};
        }
        if (s == 0) {
            // the continuing instances keep T_0 unchanged
            std::swap(P.T, P.Tnew);
            P.T.n = roff[Kn];
            P.T.nnz = seg[Kn];
        }
        Ka = Kn;
        return EXPM_OK;
    };
    CHK(finish(0));
    for (int s = 1; s <= maxN && Ka > 0; ++s) {
        const int64_t R = roff[Ka];
        CsrView Tv{R, (const int64_t *)P.T.rp.p, (const int32_t *)P.T.ci.p,
                   (const double *)P.T.v.p};
        int64_t cand;
        // 16 x 16 tiles on the matrix cores once the stacked iterate fills
        // its tiles (cross-instance slots are exact zeros and drop out)
        bool tiles = false;
        if (tiles_allowed(P, R)) {
            double fill = 0.0;
            CHK(bsr_pattern(P, Tv, P.T.nnz, P.tsT, &fill));
            tiles = P.tsT.ntiles > 0 && P.tsT.ntiles < INT32_MAX && fill >= P.bsr_min_fill;
        }
        if (tiles)
            CHK(tile_candidates(P, Tv, &cand));
        else
            CHK(spgemm(P, Tv, P.T.nnz, Tv, 2.0, 1.0, true, &cand));
        HIPCHK(segment_sums((const double *)P.rowsq.p, (const int64_t *)B.rowoff.p, Ka,
                            (double *)B.norm2.p, st));
        for (int k = 0; k < Ka; ++k) {
            egs[k] = A[k].a * ldexp(A[k].r0, s);
            modes[k] = 0;
            addi[k] = A[k].N == s;
        }
        HIPCHK(hipMemcpyAsync(B.egs.p, egs.data(), sizeof(double) * Ka, hipMemcpyHostToDevice,
                              st));
        HIPCHK(hipMemcpyAsync(B.modes.p, modes.data(), sizeof(int) * Ka, hipMemcpyHostToDevice,
                              st));
        HIPCHK(hipMemcpyAsync(B.addi.p, addi.data(), sizeof(int) * Ka, hipMemcpyHostToDevice,
                              st));
        HIPCHK(filter_init_batched((FilterCtl *)B.ctl.p, Ka, (const double *)B.egs.p,
                                   (const double *)B.norm2.p, (const int *)B.modes.p, P.opts.e_r,
                                   P.opts.max_filter_iter, st));
        CHK(batched_filter(P, B, Ka, R, (const int *)B.addi.p, hctl));
        HIPCHK(gather_offsets((const int64_t *)P.krp.p, (const int64_t *)B.rowoff.p, Ka,
                              (int64_t *)B.segoff.p, st));
        HIPCHK(hipMemcpyAsync(seg.data(), B.segoff.p, sizeof(int64_t) * (Ka + 1),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        CHK(ensure_csr(P, P.Tnew, R, seg[Ka]));
        HIPCHK(hipMemcpyAsync(P.Tnew.rp.p, P.krp.p, sizeof(int64_t) * (R + 1),
                              hipMemcpyDeviceToDevice, st));
        HIPCHK(write_kept((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                          (const double *)P.cv.p, R, (const FilterCtl *)B.ctl.p, 0,
                          (const int64_t *)P.Tnew.rp.p, (int32_t *)P.Tnew.ci.p,
                          (double *)P.Tnew.v.p, st, (const int32_t *)B.rowinst.p,
                          (const int *)B.addi.p));
        // finished instances: extract; the rest continue on the prefix
        int Kn = Ka;
        while (Kn > 0 && A[Kn - 1].N == s) --Kn;
        for (int k = Kn; k < Ka; ++k) {
            const int64_t nk = A[k].n, ek = seg[k + 1] - seg[k];
            int64_t *rp = (int64_t *)out_alloc(P, sizeof(int64_t) * (nk + 1));
            int32_t *ci = (int32_t *)out_alloc(P, sizeof(int32_t) * ek);
            double *v = (double *)out_alloc(P, sizeof(double) * ek);
            if (!rp || !ci || !v) return fail(EXPM_ENOMEM, "cannot allocate output");
            HIPCHK(extract_block((const int64_t *)P.Tnew.rp.p, (const int32_t *)P.Tnew.ci.p,
                                 (const double *)P.Tnew.v.p, roff[k], nk, rp, ci, v, st));
            E[A[k].idx] = expm_csr{nk, ek, rp, ci, v};
        }
        std::swap(P.T, P.Tnew);
        P.T.nnz = seg[Kn];
        Ka = Kn;
    }
    // statistics: the instance the caller passed last
    for (int k = 0; k < K; ++k) {
        if (A[k].idx != count - 1) continue;
        expm_stats &S = P.stats;
        S.M = A[k].M;
        S.N = A[k].N;
        S.normal = A[k].normal;
        S.a = A[k].a;
        S.norm_h = A[k].nh;
        S.h0 = ldexp(A[k].nh, -A[k].N);
        S.r0 = A[k].r0;
        S.eg0 = A[k].eg0;
        S.taylor_terms = A[k].terms;
        S.squarings = A[k].N;
        S.nnz_e = E[count - 1].nnz;
    }
    return EXPM_OK;
}

}  // namespace
}  // namespace host
}  // namespace xpm

extern "C" int expm_sparse_batched(expm_plan_t p, int count, const expm_csr_cview *H,
                                   const double *eps, expm_csr *E) {
    using namespace xpm::host;
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    BatchBufs B;
    collect_forward(*p);
    p->kt_used = 0;
    p->kt_kind.clear();
    // large instances (n >= opts.batch_solo_n) run on their own after the
    // stacked pass of the others
    std::vector<int> solo, stack;
    for (int k = 0; k < count && H && eps && E; ++k)
        (p->opts.batch_solo_n > 0 && H[k].n >= p->opts.batch_solo_n ? solo : stack).push_back(k);
    int s;
    if (solo.empty()) {
        s = batched(*p, B, count, H, eps, E);
    } else {
        for (int k = 0; k < count; ++k) memset(&E[k], 0, sizeof E[k]);
        std::vector<expm_csr_cview> hs;
        std::vector<double> es;
        for (int k : stack) {
            hs.push_back(H[k]);
            es.push_back(eps[k]);
        }
        std::vector<expm_csr> outs(stack.size());
        s = batched(*p, B, (int)stack.size(), hs.data(), es.data(), outs.data());
        if (s == EXPM_OK)
            for (size_t i = 0; i < stack.size(); ++i) E[stack[i]] = outs[i];
        else
            for (expm_csr &o : outs) {
                out_free(*p, o.rowptr);
                out_free(*p, o.col);
                out_free(*p, o.val);
            }
        for (size_t i = 0; s == EXPM_OK && i < solo.size(); ++i) {
            s = forward(*p, &H[solo[i]], eps[solo[i]], &E[solo[i]]);
            if (s != EXPM_OK) s = fail(s, "instance %d: %s", solo[i], g_err.c_str());
        }
        free_adjoint_state(*p);   // no adjoint follows a batched call
    }
    free_bufs(*p, B);
    if (s == EXPM_OK && light_profile(*p)) {
        (void)hipStreamSynchronize(p->st);
        ktimer_collect(*p);
    }
    if (s != EXPM_OK) {
        (void)hipStreamSynchronize(p->st);
        (void)hipGetLastError();
        for (int k = 0; E && k < count; ++k) {
            out_free(*p, E[k].rowptr);
            out_free(*p, E[k].col);
            out_free(*p, E[k].val);
            memset(&E[k], 0, sizeof E[k]);
        }
        p->stats.status = s;
    } else {
        p->have_stats = true;
    }
    return s;
}
