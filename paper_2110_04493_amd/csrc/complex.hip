// Algorithm 4.2 for a complex H (the paper states the method for H in
// C^{n x n}; section 4, problem (4.20)): the same steps as the real forward
// with complex values, a (real, imaginary) pair of doubles per entry.
//
//   steps 1-3  ||H||_F, (M, N) by problem (4.20), the normality test of
//              step 2 with the conjugate transpose (H H^* = H^* H; exactly
//              Hermitian or skew-Hermitian H is normal without it), a, r0,
//              the Taylor budget; H0 = H 2^-N;
//   Taylor     S_i = filter(S_{i-1} H0 / i), T_0 = S_1 + ... + S_M' added
//              term after term (Eq. (4.10)-(4.14));
//   step 4     T <- filter(2T + T T) against a r_i ||I + T~||_F (Eq. (4.15));
//   step 5     E = I + T_N.
//
// Algorithm 4.1 runs on the moduli |z|.  Every product runs on scalar rows
// (the row Gustavson kernels with two accumulators per slot); there is no
// locality reordering, tile path or adjoint for complex inputs.
#include <limits.h>
#include <math.h>
#include <string.h>

#include "plan.hpp"

namespace xpm {
namespace host {

namespace {

// dst = A + B (complex, exact zeros dropped).
int add_z(expm_plan_s &P, const DCsr &A, const DCsr &B, DCsr &dst) {
    const int64_t n = A.n;
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure_csr(P, dst, n, A.nnz + B.nnz, 2));
    HIPCHK(add_count_z(A.view(), B.view(), (int64_t *)P.cnt.p, P.st));
    CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)dst.rp.p, n));
    HIPCHK(add_write_z(A.view(), B.view(), (const int64_t *)dst.rp.p, (int32_t *)dst.ci.p,
                       (double *)dst.v.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, (int64_t *)dst.rp.p + n, sizeof(int64_t),
                          hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    memcpy(&dst.nnz, P.host, sizeof(int64_t));
    return EXPM_OK;
}

// The candidate of the last product as a standalone complex CSR.
int take_candidate(expm_plan_s &P, int64_t n, int64_t cand, DCsr &dst) {
    CHK(ensure_csr(P, dst, n, cand, 2));
    HIPCHK(hipMemcpyAsync(dst.rp.p, P.crp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                          P.st));
    HIPCHK(hipMemcpyAsync(dst.ci.p, P.cci.p, sizeof(int32_t) * cand, hipMemcpyDeviceToDevice,
                          P.st));
    HIPCHK(hipMemcpyAsync(dst.v.p, P.cv.p, sizeof(double) * 2 * cand, hipMemcpyDeviceToDevice,
                          P.st));
    return EXPM_OK;
}

// ||X||_F^2 of a complex matrix with m stored entries, read back.
int sumsq_z(expm_plan_s &P, const DCsr &X, int64_t m, double *out) {
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    HIPCHK(sumsq((const double *)X.v.p, nullptr, 2 * m, (double *)P.part.p, kParts,
                 (double *)P.norm2.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.norm2.p, sizeof(double), hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    memcpy(out, P.host, sizeof(double));
    return EXPM_OK;
}

// Algorithm 4.2 step 2 over C: exactly Hermitian or skew-Hermitian H is
// normal; otherwise ||H H^* - H^* H||_F <= 16 u ||H||_F^2 decides.
int detect_normal_z(expm_plan_s &P, const DCsr &H, double nh, int *normal) {
    const int64_t n = H.n;
    DCsr Hp, Hs, X, Y, Z;
    auto free_all = at_exit([&] {
        release(P, Hp);
        release(P, Hs);
        release(P, X);
        release(P, Y);
        release(P, Z);
    });
    // H^*: the transposed pattern with each entry's position in H, then the
    // conjugated values gathered through the positions
    CHK(transpose_pos(P, H, Hp));
    CHK(ensure_csr(P, Hs, n, H.nnz, 2));
    HIPCHK(hipMemcpyAsync(Hs.rp.p, Hp.rp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                          P.st));
    HIPCHK(hipMemcpyAsync(Hs.ci.p, Hp.ci.p, sizeof(int32_t) * H.nnz, hipMemcpyDeviceToDevice,
                          P.st));
    HIPCHK(gather_conj_z((const double *)H.v.p, (const int64_t *)Hp.v.p, H.nnz,
                         (double *)Hs.v.p, P.st));
    CHK(ensure(P, P.flags, sizeof(int) * 4));
    const int ones[3] = {1, 1, 1};
    HIPCHK(hipMemcpyAsync(P.flags.p, ones, sizeof ones, hipMemcpyHostToDevice, P.st));
    HIPCHK(compare_csr_z(H.view(), Hs.view(), H.nnz, (int *)P.flags.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.flags.p, sizeof(int) * 3, hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    int f[3];
    memcpy(f, P.host, sizeof f);
    if (f[0] && (f[1] || f[2])) {
        *normal = 1;
        return EXPM_OK;
    }
    int64_t c1, c2;
    CHK(spgemm(P, H.view(), H.nnz, Hs.view(), 0.0, 1.0, false, &c1, true));
    CHK(take_candidate(P, n, c1, X));
    CHK(spgemm(P, Hs.view(), Hs.nnz, H.view(), 0.0, 1.0, false, &c2, true));
    CHK(take_candidate(P, n, c2, Y));
    HIPCHK(negate_values((double *)Y.v.p, 2 * c2, P.st));
    CHK(add_z(P, X, Y, Z));   // H H^* - H^* H
    double c;
    CHK(sumsq_z(P, Z, Z.nnz, &c));
    *normal = sqrt(c) <= 16.0 * ldexp(1.0, -53) * nh * nh;
    return EXPM_OK;
}

}  // namespace

int forward_z(expm_plan_s &P, const expm_csr_cview *Hv, double eps, expm_csr *E) {
    CHK(check_view(Hv));
    if (!E) return fail(EXPM_EINVAL, "E is NULL");
    memset(E, 0, sizeof *E);
    if (!(eps >= ldexp(1.0, -60) && eps < 1.0))
        return fail(EXPM_EINVAL, "eps = %g outside [2^-60, 1)", eps);
    if (P.arena) return fail(EXPM_ENOTIMPL, "complex inputs run with device allocation only");
    if (P.opts.filter_mode == EXPM_FILTER_FIXED_REL)
        return fail(EXPM_ENOTIMPL, "the FPIM's fixed filter is not provided for complex H");
    if (P.opts.norm != EXPM_NORM_FRO)
        return fail(EXPM_ENOTIMPL, "complex H takes the Frobenius norm only");
    hipStream_t st = P.st;
    const int64_t n = Hv->n, nnz = Hv->nnz;
    free_adjoint_state(P);   // no adjoint follows a complex call
    memset(&P.stats, 0, sizeof P.stats);
    P.have_stats = false;
    P.perm_active = false;
    P.peak = P.live;
    expm_stats &S = P.stats;
    for (int i = 0; i < EXPM_MAXSTEP; ++i) S.sq_band[i] = -1;
    if (n == 0) {
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, 0, 0, &rp, &ci, &v, 2));
        out_free(P, ci);
        out_free(P, v);
        HIPCHK(hipMemsetAsync(rp, 0, sizeof(int64_t), st));
        E->rowptr = rp;
        P.have_stats = true;
        return EXPM_OK;
    }
    TraceRange phase("expm_z plan (steps 1-3)");
    // H to the workspace, checked, and ||H||_F
    DCsr &H0 = P.H0;
    const hipMemcpyKind kind = Hv->on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CHK(ensure_csr(P, H0, n, nnz, 2));
    HIPCHK(hipMemcpyAsync(H0.rp.p, Hv->rowptr, sizeof(int64_t) * (n + 1), kind, st));
    if (nnz) {
        HIPCHK(hipMemcpyAsync(H0.ci.p, Hv->col, sizeof(int32_t) * nnz, kind, st));
        HIPCHK(hipMemcpyAsync(H0.v.p, Hv->val, sizeof(double) * 2 * nnz, kind, st));
    }
    CHK(ensure(P, P.flags, sizeof(int) * 4));
    HIPCHK(hipMemsetAsync(P.flags.p, 0, sizeof(int), st));
    HIPCHK(validate_csr(H0.view(), nnz, (int *)P.flags.p, st));
    HIPCHK(check_finite((const double *)H0.v.p, 2 * nnz, (int *)P.flags.p, st));
    HIPCHK(hipMemcpyAsync((char *)P.host + 64, P.flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    double nh2;
    CHK(sumsq_z(P, H0, nnz, &nh2));
    int flag;
    memcpy(&flag, (char *)P.host + 64, sizeof flag);
    if (flag & 1) return fail(EXPM_EINVAL, "rowptr is not a valid CSR row pointer");
    if (flag & 2) return fail(EXPM_EINVAL, "column indices out of range or not strictly increasing");
    if (flag & 4) return fail(EXPM_EINVAL, "H holds NaN or Inf");
    const double nh = sqrt(nh2);
    S.norm_h = nh;
    if (nh == 0.0) {   // e^0 = I
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, n, n, &rp, &ci, &v, 2));
        HIPCHK(fill_identity_z(n, rp, ci, v, st));
        E->n = n;
        E->nnz = n;
        E->rowptr = rp;
        E->col = ci;
        E->val = v;
        S.normal = 1;
        S.nnz_e = n;
        P.have_stats = true;
        return EXPM_OK;
    }
    int M, N;
    const int s = plan_mn(nh, eps, &M, &N);
    if (s == EXPM_ERANGE) return fail(EXPM_ERANGE, "no (M, N) satisfies problem (4.20)");
    if (s) return fail(s, "invalid norm %g", nh);
    if (N >= EXPM_MAXSTEP - 1 || M >= EXPM_MAXSTEP - 1)
        return fail(EXPM_ERANGE, "(M, N) = (%d, %d) exceeds the step limit", M, N);
    int normal = P.opts.normal;
    if (normal < 0) CHK(detect_normal_z(P, H0, nh, &normal));
    double a = 1.0 / (N + 1);
    if (!normal && (P.opts.literal_a || 1.0 / nh < a)) a = 1.0 / nh;
    if (P.opts.filter_mode != EXPM_FILTER_PAPER) a = 0.0;
    const double h0 = ldexp(nh, -N), r0 = plan_r0(M, h0);
    const double eg0 = a * r0 / (M * exp(2.0 * h0));
    S.M = M;
    S.N = N;
    S.normal = normal;
    S.a = a;
    S.h0 = h0;
    S.r0 = r0;
    S.eg0 = eg0;
    const bool diag = P.opts.diagnostics != 0;
    if (diag) CHK(ensure(P, P.bands, sizeof(long long) * 2 * (N + 1)));
    // Locality reordering on request (reorder >= 1; the default leaves complex
    // H in its order, since the complex row products, the only complex path,
    // gain nothing from it): H' = P H P^T replaces H, and E is permuted back
    // at the end.
    {
        const int ro = P.opts.reorder;
        P.ordering = 0;
        if (ro >= 1)
            CHK(compute_reorder(P, H0.view(), nnz, ro == 2 ? 2 : 1, &P.perm_active));
        S.ordering = P.perm_active ? P.ordering : 0;
        if (P.perm_active) {
            CHK(ensure_csr(P, P.Hp, n, nnz, 2));
            CHK(permute_csr(P, H0.view(), nnz, (const int32_t *)P.order.p,
                            (const int32_t *)P.newidx.p, (int64_t *)P.Hp.rp.p,
                            (int32_t *)P.Hp.ci.p, (double *)P.Hp.v.p, nullptr, true));
            std::swap(P.H0, P.Hp);
        }
    }
    const int32_t *border = P.perm_active ? (const int32_t *)P.order.p : nullptr;

    phase.next("expm_z taylor seed");
    const auto t_taylor0 = std::chrono::steady_clock::now();
    HIPCHK(scale_ldexp((const double *)H0.v.p, (double *)H0.v.p, 2 * nnz, -N, st));
    const CsrView H0v = H0.view();
    DCsr &Sc = P.S, &Sn = P.Snew, &T = P.T, &Tn = P.Tnew;
    CHK(copy_csr(P, Sc, H0, 2));
    CHK(copy_csr(P, T, H0, 2));
    S.taylor_terms = 1;
    for (int i = 2; i <= M; ++i) {
        int64_t cand, kept;
        CHK(spgemm(P, Sc.view(), Sc.nnz, H0v, 0.0, (double)i, false, &cand, true));
        FilterCtl h{};
        CHK(filter_and_count(P, n, cand, eg0, nullptr, false, 0.0, false, &h, &kept, true));
        S.taylor_theta[i] = h.theta;
        S.taylor_iters[i] = h.iter;
        S.taylor_cand[i] = cand;
        S.taylor_kept[i] = kept;
        if (kept == 0) break;   // later terms are exactly zero
        CHK(write_filtered(P, n, Sn, kept, false, false, true));
        Sn.nnz = kept;
        std::swap(Sc, Sn);
        CHK(add_z(P, T, Sc, Tn));   // T_0 += S_i
        std::swap(T, Tn);
        S.taylor_terms = i;
    }
    S.t_taylor_ms = ms_since(t_taylor0);
    if (diag) HIPCHK(band_of(T.view(), border, (long long *)P.bands.p, st));

    phase.next("expm_z squarings");
    double ri = r0;
    for (int i = 1; i <= N; ++i) {
        ri = P.opts.exact_ri ? 2.0 * ri + ri * ri : ldexp(r0, i);
        S.sq_ri[i] = ri;
        int64_t cand, kept;
        CHK(spgemm(P, T.view(), T.nnz, T.view(), 2.0, 1.0, true, &cand, true));
        CHK(ensure(P, P.norm2, sizeof(double) * 2));
        CHK(ensure(P, P.part, sizeof(double) * kParts));
        HIPCHK(sum_values((const double *)P.rowsq.p, n, (double *)P.part.p, kParts,
                          (double *)P.norm2.p, st));
        FilterCtl h{};
        CHK(filter_and_count(P, n, cand, a * ri, (const double *)P.norm2.p, false, 0.0, false, &h,
                             &kept, true));
        CHK(write_filtered(P, n, Tn, kept, false, false, true));
        Tn.nnz = kept;
        if (P.opts.profile == 1 && P.have_events) {
            // phase times of the step (symbolic, numeric, filter and
            // compaction) and its partial products, as for real H
            HIPCHK(hipEventRecord(P.ev[3], st));
            HIPCHK(hipEventSynchronize(P.ev[3]));
            float t0, t1, t2;
            HIPCHK(hipEventElapsedTime(&t0, P.ev[0], P.ev[1]));
            HIPCHK(hipEventElapsedTime(&t1, P.ev[1], P.ev[2]));
            HIPCHK(hipEventElapsedTime(&t2, P.ev[2], P.ev[3]));
            S.t_sym_ms[i] = t0;
            S.t_num_ms[i] = t1;
            S.t_filter_ms[i] = t2;
            S.sq_fma[i] = P.last_fma;
            S.sq_in[i] = T.nnz;
        }
        std::swap(T, Tn);
        if (diag) HIPCHK(band_of(T.view(), border, (long long *)P.bands.p + 2 * i, st));
        S.sq_theta[i] = h.theta;
        S.sq_iters[i] = h.iter;
        S.sq_cand[i] = cand;
        S.sq_kept[i] = kept;
        S.sq_budget[i] = h.eg;
        S.sq_normF[i] = a * ri > 0.0 ? h.eg / (a * ri) : 0.0;
        S.sq_dropped[i] = h.b;
        S.sq_tiles[i] = 0;
    }
    S.squarings = N;

    phase.next("expm_z finish (E = I + T_N)");
    {
        // T_N is the candidate of the compaction that adds the identity
        std::swap(P.crp, T.rp);
        std::swap(P.cci, T.ci);
        std::swap(P.cv, T.v);
        auto swap_back = at_exit([&] {
            std::swap(P.crp, T.rp);
            std::swap(P.cci, T.ci);
            std::swap(P.cv, T.v);
        });
        FilterCtl h{};
        int64_t kept;
        CHK(filter_and_count(P, n, T.nnz, 0.0, nullptr, true, -1.0, true, &h, &kept, true));
        int64_t *rp;
        int32_t *ci;
        double *v;
        CHK(alloc_output(P, n, kept, &rp, &ci, &v, 2));
        // E' (the reordered result) goes to the workspace and is permuted
        // back into the caller's order; without reordering E is written
        // directly
        int64_t *erp = rp;
        int32_t *eci = ci;
        double *ev = v;
        if (P.perm_active) {
            CHK(ensure_csr(P, P.Eperm, n, kept, 2));
            erp = (int64_t *)P.Eperm.rp.p;
            eci = (int32_t *)P.Eperm.ci.p;
            ev = (double *)P.Eperm.v.p;
        }
        HIPCHK(hipMemcpyAsync(erp, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                              st));
        HIPCHK(write_kept_z((const int64_t *)P.crp.p, (const int32_t *)P.cci.p,
                            (const double *)P.cv.p, n, (const FilterCtl *)P.ctl.p, 1, erp, eci,
                            ev, st));
        if (P.perm_active)
            CHK(permute_csr(P, P.Eperm.view(), kept, (const int32_t *)P.newidx.p,
                            (const int32_t *)P.order.p, rp, ci, v, nullptr, true));
        E->n = n;
        E->nnz = kept;
        E->rowptr = rp;
        E->col = ci;
        E->val = v;
        S.nnz_e = kept;
    }
    if (diag) {   // l(T^_i) = l1 + l2 of Eq. (3.1), 0 for an empty iterate
        long long *hb = (long long *)P.host;
        HIPCHK(hipMemcpyAsync(hb, P.bands.p, sizeof(long long) * 2 * (N + 1),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        for (int i = 0; i <= N; ++i)
            S.sq_band[i] = hb[2 * i] == LLONG_MIN ? 0 : hb[2 * i] + hb[2 * i + 1];
    }
    S.peak_workspace_bytes = P.peak;
    P.have_stats = true;
    return EXPM_OK;
}

}  // namespace host
}  // namespace xpm

using namespace xpm::host;

extern "C" int expm_sparse_z(expm_plan_t p, const expm_csr_cview *H, double eps, expm_csr *E) {
    g_err.clear();
    if (!p) return fail(EXPM_EINVAL, "plan is NULL");
    collect_forward(*p);
    const auto t0 = std::chrono::steady_clock::now();
    const int s = forward_z(*p, H, eps, E);
    if (s == EXPM_OK) p->stats.t_total_ms = ms_since(t0);   // host time of the call
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
