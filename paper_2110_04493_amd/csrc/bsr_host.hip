// Host drivers of the 16 x 16 tile squaring step and its adjoint (kernels in
// bsr.hip and bsr_adjoint.hip).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "plan.hpp"

namespace xpm {
namespace host {

void release(expm_plan_s &P, TileSet &ts) {
    Buf *all[] = {&ts.lo, &ts.words, &ts.woff, &ts.rt,   &ts.cnt, &ts.tb,
                  &ts.tA, &ts.tB,    &ts.cols, &ts.rows, &ts.seg, &ts.mir};
    for (Buf *b : all) release(P, *b);
    ts.nb = ts.ntiles = 0;
}

// Tile pattern of T (origin, bit maps with prefix counts, tile bases) and
// C's tile pattern counts for C = 2T + T*T from T's tile pattern ts: per
// block row the origin and bit-map words (P.c_lo, P.c_words, P.c_woff) and
// the tile counts (P.c_cnt, P.c_tb); the totals are c_woff[nb], c_tb[nb].
static int c_pattern_count(expm_plan_s &P, const TileSet &ts, int64_t n) {
    hipStream_t st = P.st;
    const int64_t nb = ts.nb;
    CHK(ensure(P, P.c_lo, sizeof(int32_t) * (nb + 1)));
    CHK(ensure(P, P.c_words, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.c_woff, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.c_cnt, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.c_tb, sizeof(int64_t) * (nb + 1)));
    const int32_t *lo = (const int32_t *)ts.lo.p;
    const int64_t *woff = (const int64_t *)ts.woff.p, *tb = (const int64_t *)ts.tb.p;
    const uint2 *rt = (const uint2 *)ts.rt.p;
    HIPCHK(bsr_cbounds(nb, lo, woff, rt, tb, (int32_t *)P.c_lo.p, (int64_t *)P.c_words.p, st));
    CHK(scan(P, (const int64_t *)P.c_words.p, (int64_t *)P.c_woff.p, nb));
    HIPCHK(bsr_cpattern(n, nb, lo, woff, rt, (const int32_t *)P.c_lo.p,
                        (const int64_t *)P.c_woff.p, (int64_t *)P.c_cnt.p, nullptr, nullptr,
                        nullptr, st));
    CHK(scan(P, (const int64_t *)P.c_cnt.p, (int64_t *)P.c_tb.p, nb));
    return EXPM_OK;
}

// T's fill: stored entries over tile slots.  With with_c, the counts of the
// product's tile pattern are taken too and read back with T's tile count
// (one wait instead of two), for the tile_product call that follows.
int bsr_pattern(expm_plan_s &P, CsrView T, int64_t nnz, TileSet &ts, double *fill,
                bool with_c) {
    hipStream_t st = P.st;
    P.c_pre = false;
    const int64_t n = T.n, nb = (n + 15) / 16;
    ts.nb = nb;
    CHK(ensure(P, ts.lo, sizeof(int32_t) * (nb + 1)));
    CHK(ensure(P, ts.words, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, ts.woff, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, ts.cnt, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, ts.tb, sizeof(int64_t) * (nb + 1)));
    HIPCHK(bsr_bounds(T, nb, (int32_t *)ts.lo.p, (int64_t *)ts.words.p, st));
    CHK(scan(P, (const int64_t *)ts.words.p, (int64_t *)ts.woff.p, nb));
    int64_t *hl = (int64_t *)P.host;
    // a block row's bit map spans at most (nb + 31) / 32 + 1 words: when that
    // bound is small the rank table is sized by it, saving a readback
    const int64_t bound = nb * ((nb + 31) / 32 + 1);
    int64_t words = bound;
    if (bound * (int64_t)sizeof(uint2) > ((int64_t)64 << 20)) {
        HIPCHK(hipMemcpyAsync(hl, (int64_t *)ts.woff.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        words = hl[0];
    }
    CHK(ensure(P, ts.rt, sizeof(uint2) * (words + 1)));
    HIPCHK(bsr_bitmap(T, nb, (const int32_t *)ts.lo.p, (const int64_t *)ts.woff.p,
                      (uint2 *)ts.rt.p, (int64_t *)ts.cnt.p, st));
    CHK(scan(P, (const int64_t *)ts.cnt.p, (int64_t *)ts.tb.p, nb));
    if (with_c) CHK(c_pattern_count(P, ts, n));
    HIPCHK(hipMemcpyAsync(hl, (int64_t *)ts.tb.p + nb, sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    if (with_c) {
        HIPCHK(hipMemcpyAsync(hl + 1, (int64_t *)P.c_tb.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hl + 2, (int64_t *)P.c_woff.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
    }
    CHK(sync(P));
    ts.ntiles = hl[0];
    if (with_c) {
        P.c_pre = true;
        P.c_pre_tiles = hl[1];
        P.c_pre_words = hl[2];
    }
    CHK(ensure(P, ts.cols, sizeof(int32_t) * (ts.ntiles + 1)));
    CHK(ensure(P, ts.rows, sizeof(int32_t) * (ts.ntiles + 1)));
    HIPCHK(bsr_tcols(nb, (const int32_t *)ts.lo.p, (const int64_t *)ts.woff.p,
                     (const uint2 *)ts.rt.p, (const int64_t *)ts.tb.p, (int32_t *)ts.cols.p,
                     (int32_t *)ts.rows.p, st));
    *fill = ts.ntiles ? (double)nnz / ((double)ts.ntiles * 256.0) : 0.0;
    return EXPM_OK;
}

// T's values as tiles of the pattern, in both operand layouts (with b_only,
// for a symmetric T, the B layout and each tile's mirror index): a table of
// row segments, then every tile assembled whole.
int bsr_tiles(expm_plan_s &P, CsrView T, TileSet &ts, bool b_only) {
    const size_t nt = (size_t)(ts.ntiles > 0 ? ts.ntiles : 1);
    ts.b_only = b_only;
    if (b_only) {
        // symmetric T: the A layout of tile (I, K) is the B layout of (K, I)
        CHK(ensure(P, ts.mir, sizeof(int64_t) * nt));
        CHK(ensure(P, P.mirror_bad, sizeof(int)));
        HIPCHK(bsr_tile_mirrors(ts.ntiles, (const int32_t *)ts.lo.p, (const int64_t *)ts.woff.p,
                                (const uint2 *)ts.rt.p, (const int64_t *)ts.tb.p,
                                (const int32_t *)ts.cols.p, (const int32_t *)ts.rows.p,
                                (int64_t *)ts.mir.p, (int *)P.mirror_bad.p, P.st));
    } else {
        CHK(ensure(P, ts.tA, sizeof(double) * 256 * nt));
    }
    CHK(ensure(P, ts.tB, sizeof(double) * 256 * nt));
    CHK(ensure(P, ts.seg, sizeof(int64_t) * 16 * nt));
    HIPCHK(hipMemsetAsync(ts.seg.p, 0, sizeof(int64_t) * 16 * nt, P.st));
    HIPCHK(bsr_seg(T, (const int32_t *)ts.lo.p, (const int64_t *)ts.woff.p,
                   (const uint2 *)ts.rt.p, (const int64_t *)ts.tb.p, (int64_t *)ts.seg.p, P.st));
    HIPCHK(bsr_assemble(T, ts.ntiles, (const int32_t *)ts.cols.p, (const int32_t *)ts.rows.p,
                        (const int64_t *)ts.seg.p, b_only ? nullptr : (double *)ts.tA.p,
                        (double *)ts.tB.p, P.st));
    return EXPM_OK;
}

// C = 2T + T*T on tiles (T's pattern already in P.tsT): T's tiles, C's tile
// pattern (rank table, panels) and the candidate tiles in P.c_tiles; the
// product kernel is bracketed by events ev[1], ev[2] when prof.  With
// tile_norms the product also leaves each tile's share of ||I + T~||_F^2 and
// its nonzero count in P.c_sq / P.c_nz.  *ctiles_out receives the number of
// candidate tiles.
int tile_product(expm_plan_s &P, CsrView T, bool prof, bool tile_norms, int64_t *ctiles_out,
                 bool upper) {
    hipStream_t st = P.st;
    TileSet &ts = P.tsT;
    const int64_t n = T.n, nb = ts.nb;
    int64_t *hl = (int64_t *)P.host;
    if (upper) {   // flags a pattern found unsymmetric (T's tiles or C's)
        CHK(ensure(P, P.mirror_bad, sizeof(int)));
        HIPCHK(hipMemsetAsync(P.mirror_bad.p, 0, sizeof(int), st));
    }
    CHK(bsr_tiles(P, T, ts, upper));
    // C's tile pattern (its counts already read back by bsr_pattern when it
    // ran with with_c just before)
    const int32_t *lo = (const int32_t *)ts.lo.p;
    const int64_t *woff = (const int64_t *)ts.woff.p, *tb = (const int64_t *)ts.tb.p;
    const uint2 *rt = (const uint2 *)ts.rt.p;
    int64_t ctiles, cwords;
    if (P.c_pre) {
        ctiles = P.c_pre_tiles;
        cwords = P.c_pre_words;
        P.c_pre = false;
    } else {
        CHK(c_pattern_count(P, ts, n));
        HIPCHK(hipMemcpyAsync(hl, (int64_t *)P.c_tb.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hl + 2, (int64_t *)P.c_woff.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        CHK(sync(P));
        ctiles = hl[0];
        cwords = hl[2];
    }
    CHK(ensure(P, P.c_cols, sizeof(int32_t) * (ctiles + 1)));
    CHK(ensure(P, P.c_tiles, sizeof(double) * 256 * (size_t)(ctiles + 1)));
    CHK(ensure(P, P.c_rt, sizeof(uint2) * (cwords + 1)));
    if (tile_norms) {
        CHK(ensure(P, P.c_sq, sizeof(double) * (ctiles + 1)));
        CHK(ensure(P, P.c_nz, sizeof(int32_t) * (ctiles + 1)));
        CHK(ensure(P, P.c_mn, sizeof(double) * (ctiles + 1)));
        CHK(ensure(P, P.c_mx, sizeof(double) * (ctiles + 1)));
        CHK(ensure(P, P.c_rc, sizeof(uint4) * (ctiles + 1)));
        CHK(ensure(P, P.c_kc, sizeof(uint4) * (ctiles + 1)));
        CHK(ensure(P, P.b_dg, sizeof(double) * (nb + 1)));
    }
    HIPCHK(bsr_cpattern(n, nb, lo, woff, rt, (const int32_t *)P.c_lo.p,
                        (const int64_t *)P.c_woff.p, (int64_t *)P.c_cnt.p,
                        (const int64_t *)P.c_tb.p, (int32_t *)P.c_cols.p, (uint2 *)P.c_rt.p,
                        st));
    {
        // panels of four block rows and their shared column groups
        const int64_t np = (nb + 3) / 4;
        CHK(ensure(P, P.p_lo, sizeof(int32_t) * (np + 1)));
        CHK(ensure(P, P.p_words, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_woff, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_cnt, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_ofs, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_gcnt, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_gofs, sizeof(int64_t) * (np + 1)));
        CHK(ensure(P, P.p_cols, sizeof(int32_t) * (ctiles + 1)));
        const int32_t *clo = (const int32_t *)P.c_lo.p;
        const int64_t *cwoff = (const int64_t *)P.c_woff.p;
        HIPCHK(bsr_panel_bounds(nb, clo, cwoff, (int32_t *)P.p_lo.p, (int64_t *)P.p_words.p, st));
        CHK(scan(P, (const int64_t *)P.p_words.p, (int64_t *)P.p_woff.p, np));
        HIPCHK(bsr_panel_cols(n, nb, clo, cwoff, (const uint2 *)P.c_rt.p,
                              (const int32_t *)P.p_lo.p, (const int64_t *)P.p_woff.p,
                              (int64_t *)P.p_cnt.p, nullptr, nullptr, st, upper));
        CHK(scan(P, (const int64_t *)P.p_cnt.p, (int64_t *)P.p_ofs.p, np));
        HIPCHK(bsr_panel_cols(n, nb, clo, cwoff, (const uint2 *)P.c_rt.p,
                              (const int32_t *)P.p_lo.p, (const int64_t *)P.p_woff.p,
                              (int64_t *)P.p_cnt.p, (const int64_t *)P.p_ofs.p,
                              (int32_t *)P.p_cols.p, st, upper));
        HIPCHK(bsr_panel_groups((const int64_t *)P.p_cnt.p, nb, (int64_t *)P.p_gcnt.p, st));
        CHK(scan(P, (const int64_t *)P.p_gcnt.p, (int64_t *)P.p_gofs.p, np));
        CHK(ensure(P, P.p_owner, sizeof(int32_t) * (bsr_panel_work_bound(ctiles, nb) + 1)));
        HIPCHK(work_owner((const int64_t *)P.p_gofs.p, np, (int32_t *)P.p_owner.p, st));
        // launched on a bound of the work-item count (a panel's union holds
        // at most the sum of its rows' tiles); the kernel reads the exact
        // count, p_gofs[np], and surplus workgroups return at once
    }
    const int64_t nwork = bsr_panel_work_bound(ctiles, nb);
    if (upper && tile_norms) CHK(ensure(P, P.c_mir, sizeof(int64_t) * (ctiles + 1)));
    if (prof) HIPCHK(hipEventRecord(P.ev[1], st));
    if (light_profile(P)) CHK(ktimer_mark(P, 0));
    HIPCHK(bsr_numeric_panel(nb, lo, woff, rt, tb, (const int32_t *)ts.cols.p,
                             (const double *)ts.tA.p, (const double *)ts.tB.p,
                             (const int64_t *)P.p_gofs.p, (const int64_t *)P.p_gofs.p + (nb + 3) / 4,
                             (const int32_t *)P.p_owner.p,
                             (const int64_t *)P.p_ofs.p, (const int32_t *)P.p_cols.p,
                             (const int32_t *)P.c_lo.p, (const int64_t *)P.c_woff.p,
                             (const uint2 *)P.c_rt.p, (const int64_t *)P.c_tb.p,
                             (double *)P.c_tiles.p, n,
                             tile_norms ? (double *)P.c_sq.p : nullptr,
                             tile_norms ? (int32_t *)P.c_nz.p : nullptr,
                             tile_norms ? (double *)P.c_mn.p : nullptr,
                             tile_norms ? (double *)P.c_mx.p : nullptr,
                             tile_norms ? (uint4 *)P.c_rc.p : nullptr,
                             tile_norms ? (double *)P.b_dg.p : nullptr, nwork, st, upper,
                             upper ? (int *)P.mirror_bad.p : nullptr,
                             upper && tile_norms ? (int64_t *)P.c_mir.p : nullptr,
                             upper ? (const int64_t *)ts.mir.p : nullptr));
    if (prof) HIPCHK(hipEventRecord(P.ev[2], st));
    if (light_profile(P)) CHK(ktimer_mark(P, 0));
    *ctiles_out = ctiles;
    return EXPM_OK;
}

// T~ = 2T + T*T on tiles, returned unfiltered as a CSR candidate in
// P.crp / P.cci / P.cv (every nonzero slot, columns sorted) with the rows'
// contributions to ||I + T~||_F^2 in P.rowsq: the same outputs as the
// scalar product, for callers that filter rows with per-row thresholds
// (the batched path).  T's pattern must already be in P.tsT.
int tile_candidates(expm_plan_s &P, CsrView T, int64_t *cand) {
    hipStream_t st = P.st;
    const int64_t n = T.n;
    int64_t ctiles = 0;
    CHK(tile_product(P, T, false, false, &ctiles));
    const int64_t *ctb = (const int64_t *)P.c_tb.p, *ccnt = (const int64_t *)P.c_cnt.p;
    const int32_t *ccols = (const int32_t *)P.c_cols.p;
    const double *ctl_tiles = (const double *)P.c_tiles.p;
    CHK(ensure(P, P.rowsq, sizeof(double) * (n + 1)));
    HIPCHK(bsr_rowsq(n, ctb, ccnt, ccols, ctl_tiles, (double *)P.rowsq.p, st));
    CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.crp, sizeof(int64_t) * (n + 1)));
    FilterCtl *ctl = (FilterCtl *)P.ctl.p;
    HIPCHK(filter_init_theta(ctl, 0.0, st));   // keep every nonzero slot
    HIPCHK(bsr_count(n, ctb, ccnt, ccols, ctl_tiles, nullptr, nullptr, nullptr, nullptr, ctl,
                     (int64_t *)P.cnt.p, st));
    CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.crp.p, n));
    int64_t *hl = (int64_t *)P.host;
    HIPCHK(hipMemcpyAsync(hl, (int64_t *)P.crp.p + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    CHK(sync(P));
    *cand = hl[0];
    CHK(ensure(P, P.cci, sizeof(int32_t) * (*cand + 1)));
    CHK(ensure(P, P.cv, sizeof(double) * (*cand + 1)));
    HIPCHK(bsr_write(n, ctb, ccnt, ccols, ctl_tiles, nullptr, ctl, (const int64_t *)P.crp.p,
                     (int32_t *)P.cci.p, (double *)P.cv.p, st));
    return EXPM_OK;
}

// One filtered squaring on tiles (T's pattern already in P.tsT): fills the
// candidate tiles, runs Algorithm 4.1 (or applies theta_fixed) and writes the
// kept entries of T~ into dst as CSR.
int square_step_bsr(expm_plan_s &P, const DCsr &T, DCsr &dst, double a_ri, bool use_fixed,
                    double theta_fixed, bool exact_alloc, int stat_i) {
    hipStream_t st = P.st;
    TileSet &ts = P.tsT;
    const int64_t n = T.n, nb = ts.nb;
    // profiling covers every launch (recomputation too); the per-step
    // statistics only the forward steps (stat_i > 0)
    const bool prof = P.opts.profile == 1 && P.have_events;
    int64_t *hl = (int64_t *)P.host;
    if (prof) {
        // algorithmic partial products of T*T (for the statistics only)
        CHK(ensure(P, P.lo, sizeof(int32_t) * n));
        CHK(ensure(P, P.words, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.ub, sizeof(int64_t) * (n + 1)));
        CHK(ensure(P, P.tmp1, sizeof(int64_t) * (n + 1)));
        HIPCHK(row_bounds(T.view(), T.view(), 1, (int32_t *)P.lo.p, (int64_t *)P.words.p,
                          (int64_t *)P.ub.p, st));
        CHK(scan(P, (const int64_t *)P.ub.p, (int64_t *)P.tmp1.p, n));
        HIPCHK(hipMemcpyAsync(hl + 16, (int64_t *)P.tmp1.p + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(P.ev[0], st));
    }
    int64_t ctiles = 0;
    // the FPIM's filter (forward steps): a threshold from the candidate's
    // 1-norm instead of Algorithm 4.1
    const bool fpim = P.fpim_eps > 0.0 && !use_fixed;
    // an exactly symmetric T (symmetric H, see forward) gives a symmetric
    // candidate: only its tiles on and right of the diagonal are formed
    const bool upper = P.sym_h;
    CHK(tile_product(P, T.view(), prof, true, &ctiles, upper));
    // ||I + T~||_F and the nonzero candidate count
    CHK(ensure(P, P.b_sq, sizeof(double) * (nb + 1)));
    CHK(ensure(P, P.b_nz, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    CHK(ensure(P, P.tmp2, sizeof(int64_t) * (nb + 1)));
    HIPCHK(bsr_norm_tiles(n, nb, (const int64_t *)P.c_tb.p, (const int64_t *)P.c_cnt.p,
                          (const int32_t *)P.c_cols.p, (const double *)P.c_sq.p,
                          (const int32_t *)P.c_nz.p, (const double *)P.b_dg.p,
                          (double *)P.b_sq.p, (int64_t *)P.b_nz.p, st));
    if (!use_fixed && !fpim)
        HIPCHK(sum_values((const double *)P.b_sq.p, nb, (double *)P.part.p, kParts,
                          (double *)P.norm2.p, st));
    CHK(scan(P, (const int64_t *)P.b_nz.p, (int64_t *)P.tmp2.p, nb));
    // Algorithm 4.1 on the tile values, then the kept counts per row
    CHK(ensure(P, P.ctl, sizeof(FilterCtl)));
    CHK(ensure(P, P.krp, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.cnt, sizeof(int64_t) * (n + 1)));
    FilterCtl *ctl = (FilterCtl *)P.ctl.p;
    if (fpim) {
        CHK(ensure(P, P.colsum, sizeof(double) * (n + 1)));
        CHK(ensure(P, P.amax, sizeof(unsigned long long) * 2));
        HIPCHK(fpim_theta_tiles(n, ctiles, (const int32_t *)P.c_cols.p,
                                (const double *)P.c_tiles.p, (double *)P.colsum.p,
                                (unsigned long long *)P.amax.p, P.fpim_eps, ctl, st));
        use_fixed = true;
    } else if (use_fixed) {
        HIPCHK(filter_init_theta(ctl, theta_fixed, st));
    } else {
        HIPCHK(filter_init(ctl, a_ri, (const double *)P.norm2.p, P.opts.e_r,
                           P.opts.max_filter_iter, st));
    }
    FilterCtl h{};
    int64_t kept = 0, cand_nz = 0;
    // the compaction's rounds of 64 candidate tiles per block row (a bound
    // of their count launches the write; it reads the exact one)
    const int64_t nround = ctiles / kWave + nb + 1;
    CHK(ensure(P, P.r_cnt, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.r_ofs, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.r_rows, sizeof(int32_t) * 16 * (nround + 1)));   // 16 rows a round
    CHK(ensure(P, P.r_owner, sizeof(int32_t) * (nround + 1)));
    HIPCHK(bsr_rounds((const int64_t *)P.c_cnt.p, nb, (int64_t *)P.r_cnt.p, st));
    CHK(scan(P, (const int64_t *)P.r_cnt.p, (int64_t *)P.r_ofs.p, nb));
    HIPCHK(work_owner((const int64_t *)P.r_ofs.p, nb, (int32_t *)P.r_owner.p, st));
    for (int round = 0;; ++round) {
        if (!use_fixed)
            for (int j = 0; j < 4; ++j)
                HIPCHK(filter_pass_tiles((const double *)P.c_tiles.p, (const double *)P.c_mn.p,
                                         (const double *)P.c_mx.p, (const double *)P.c_sq.p,
                                         ctiles, ctl, (double *)P.part.p, kParts,
                                         (uint4 *)P.c_kc.p, st,
                                         upper ? (const int64_t *)P.c_mir.p : nullptr));
        // the passes' counts hold for the final threshold only when a pass
        // ran at it: not with a fixed threshold, nor when a = 0 (then no
        // tile lies between its smallest nonzero and the threshold 0)
        HIPCHK(bsr_count(n, (const int64_t *)P.c_tb.p, (const int64_t *)P.c_cnt.p,
                         (const int32_t *)P.c_cols.p, (const double *)P.c_tiles.p,
                         (const double *)P.c_mn.p, (const double *)P.c_mx.p,
                         (const uint4 *)P.c_rc.p, use_fixed ? nullptr : (const uint4 *)P.c_kc.p,
                         ctl, (int64_t *)P.cnt.p, st, (int32_t *)P.r_rows.p,
                         (const int64_t *)P.r_ofs.p));
        CHK(scan(P, (const int64_t *)P.cnt.p, (int64_t *)P.krp.p, n));
        HIPCHK(hipMemcpyAsync(P.host, ctl, sizeof(FilterCtl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hl + 8, (int64_t *)P.krp.p + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hl + 9, (int64_t *)P.tmp2.p + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        if (upper && round == 0) {
            hl[10] = 0;
            HIPCHK(hipMemcpyAsync(hl + 10, P.mirror_bad.p, sizeof(int), hipMemcpyDeviceToHost,
                                  st));
        }
        CHK(sync(P));
        if (upper && round == 0 && (int)hl[10])
            return fail(EXPM_EHIP, "internal error: the candidate of a symmetric iterate has "
                                   "an unsymmetric tile pattern");
        memcpy(&h, P.host, sizeof h);
        kept = hl[8];
        cand_nz = hl[9];
        if (h.done) break;
        if (round > P.opts.max_filter_iter)
            return fail(EXPM_ENOTCONV, "Algorithm 4.1 did not stop");
    }
    if (h.status)
        return fail(EXPM_ENOTCONV, "Algorithm 4.1 reached %d iterations (budget %g)", h.iter,
                    h.eg);
    if (exact_alloc) release(P, dst);
    CHK(ensure_csr(P, dst, n, kept));
    HIPCHK(hipMemcpyAsync(dst.rp.p, P.krp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice,
                          st));
    HIPCHK(bsr_write_rounds(n, (const int64_t *)P.c_tb.p, (const int64_t *)P.c_cnt.p,
                            (const int32_t *)P.c_cols.p, (const double *)P.c_tiles.p,
                            (const double *)P.c_mx.p, ctl, (const int64_t *)dst.rp.p,
                            (const int32_t *)P.r_rows.p, (const int64_t *)P.r_ofs.p,
                            (const int32_t *)P.r_owner.p, nround, (int32_t *)dst.ci.p,
                            (double *)dst.v.p, st));
    expm_stats &S = P.stats;
    if (prof) {
        HIPCHK(hipEventRecord(P.ev[3], st));
        HIPCHK(hipEventSynchronize(P.ev[3]));
        float t0, t1, t2;
        HIPCHK(hipEventElapsedTime(&t0, P.ev[0], P.ev[1]));
        HIPCHK(hipEventElapsedTime(&t1, P.ev[1], P.ev[2]));
        HIPCHK(hipEventElapsedTime(&t2, P.ev[2], P.ev[3]));
        const int64_t fma = hl[16] - T.nnz;
        S.tile_launches += 1;
        S.tile_ms += t1;
        if (upper) {
            // the product forms the candidate on and right of the diagonal:
            // (fma + nnz(T)) / 2 partial products land there (a symmetric
            // pattern puts nnz(T) of them on the diagonal), with at most
            // (nnz(T) + n) / 2 entries of T added (the 2T term); it still
            // reads all of T, and writes every candidate (the transposes
            // too)
            S.tile_flops += (double)fma + (double)T.nnz + (double)T.nnz + (double)n;
            S.tile_bytes += 12.0 * (double)T.nnz + 8.0 * (double)(n + 1) +
                            12.0 * (double)cand_nz;
        } else {
            S.tile_flops += 2.0 * (double)fma + 2.0 * (double)T.nnz;
            S.tile_bytes += 12.0 * (double)T.nnz + 8.0 * (double)(n + 1) +
                            12.0 * (double)cand_nz;
        }
        if (stat_i > 0 && stat_i < EXPM_MAXSTEP) {
            S.t_sym_ms[stat_i] = t0;
            S.t_num_ms[stat_i] = t1;
            S.t_filter_ms[stat_i] = t2;
            S.sq_fma[stat_i] = fma;
            S.sq_in[stat_i] = T.nnz;
        }
    }
    if (stat_i > 0 && stat_i < EXPM_MAXSTEP) {
        S.sq_tiles[stat_i] = (int)std::min<int64_t>(ctiles, INT32_MAX);
        S.sq_theta[stat_i] = h.theta;
        S.sq_iters[stat_i] = h.iter;
        S.sq_cand[stat_i] = cand_nz;
        S.sq_kept[stat_i] = kept;
        S.sq_budget[stat_i] = fpim ? h.theta : h.eg;
        S.sq_normF[stat_i] = a_ri > 0 && !fpim ? h.eg / a_ri : 0.0;
        S.sq_dropped[stat_i] = h.b;
    }
    return EXPM_OK;
}

// The number of partial products of G T^T and T^T G (G on Tk's pattern,
// T = Tp) whose position lies in Tp's pattern, for the profile statistics:
// the masked row product run on all-ones values.
static int count_adjoint_products(expm_plan_s &P, const DCsr &Tp, const DCsr &Tk, double *pp) {
    const int64_t n = Tp.n;
    DCsr Tt;
    Buf ones_p, ones_k, cnt;
    auto free_locals = at_exit([&] {
        release(P, Tt);
        release(P, ones_p);
        release(P, ones_k);
        release(P, cnt);
    });
    CHK(transpose_csr(P, Tp, Tt));
    CHK(ensure(P, ones_p, sizeof(double) * (Tp.nnz + 1)));
    CHK(ensure(P, ones_k, sizeof(double) * (Tk.nnz + 1)));
    CHK(ensure(P, cnt, sizeof(double) * (Tp.nnz + 1)));
    HIPCHK(fill_f64((double *)ones_p.p, Tp.nnz, 1.0, P.st));
    HIPCHK(fill_f64((double *)ones_k.p, Tk.nnz, 1.0, P.st));
    const CsrView G1{n, (const int64_t *)Tk.rp.p, (const int32_t *)Tk.ci.p,
                     (const double *)ones_k.p};
    const CsrView Tt1{n, (const int64_t *)Tt.rp.p, (const int32_t *)Tt.ci.p,
                      (const double *)ones_p.p};
    const CsrView M{n, (const int64_t *)Tp.rp.p, (const int32_t *)Tp.ci.p, nullptr};
    const MaskTerm t1{G1, Tt1, 1.0}, t2{Tt1, G1, 1.0};
    CHK(masked(P, M, G1, 0.0, t1, t2, 1.0, (double *)cnt.p));
    CHK(ensure(P, P.norm2, sizeof(double) * 2));
    CHK(ensure(P, P.part, sizeof(double) * kParts));
    HIPCHK(sum_values((const double *)cnt.p, Tp.nnz, (double *)P.part.p, kParts,
                      (double *)P.norm2.p, P.st));
    HIPCHK(hipMemcpyAsync(P.host, P.norm2.p, sizeof(double), hipMemcpyDeviceToHost, P.st));
    CHK(sync(P));
    memcpy(pp, P.host, sizeof(double));
    return EXPM_OK;
}

// Adjoint squaring step on tiles.  Tp's pattern must already be in P.tsT
// (bsr_pattern); G's pattern is that of Tk.
int adjoint_step_bsr(expm_plan_s &P, const DCsr &Tp, const DCsr &Tk, const double *g,
                     double *out, bool g_pattern_ready, bool g_tiles_ready, bool want_csr,
                     bool t_tiles_ready) {
    hipStream_t st = P.st;
    TileSet &T = P.tsT, &G = P.tsG;
    const int64_t nb = T.nb;
    // a symmetric T (symmetric H) is assembled in the B layout only
    if (!t_tiles_ready) CHK(bsr_tiles(P, Tp.view(), T, P.sym_h));
    const CsrView Gv{Tk.n, (const int64_t *)Tk.rp.p, (const int32_t *)Tk.ci.p, g};
    double fg;
    if (!g_pattern_ready) CHK(bsr_pattern(P, Gv, Tk.nnz, G, &fg));
    if (!(g_pattern_ready && g_tiles_ready)) CHK(bsr_tiles(P, Gv, G));
    // T's block columns as sorted lists (T^T's block rows): for a symmetric
    // T its block rows themselves, each tile T_IK standing for its mirror
    // T_KI (the mirror index of the B-layout-only assembly)
    const int64_t *cptr;
    const int32_t *ck;
    const int64_t *ct;
    if (T.b_only) {
        cptr = (const int64_t *)T.tb.p;
        ck = (const int32_t *)T.cols.p;
        ct = (const int64_t *)T.mir.p;
    } else {
        CHK(ensure(P, P.tc_cnt, sizeof(int64_t) * (nb + 1)));
        CHK(ensure(P, P.tc_ptr, sizeof(int64_t) * (nb + 1)));
        CHK(ensure(P, P.tc_fill, sizeof(int64_t) * (nb + 1)));
        CHK(ensure(P, P.tc_k, sizeof(int32_t) * 2 * (T.ntiles + 1)));
        CHK(ensure(P, P.tc_t, sizeof(int64_t) * 2 * (T.ntiles + 1)));
        int32_t *uk = (int32_t *)P.tc_k.p, *sk = uk + (T.ntiles + 1);
        int64_t *ut = (int64_t *)P.tc_t.p, *stt = ut + (T.ntiles + 1);
        HIPCHK(hipMemsetAsync(P.tc_cnt.p, 0, sizeof(int64_t) * (nb + 1), st));
        HIPCHK(bsr_colcount(nb, (const int32_t *)T.lo.p, (const int64_t *)T.woff.p,
                            (const uint2 *)T.rt.p, (int64_t *)P.tc_cnt.p, st));
        CHK(scan(P, (const int64_t *)P.tc_cnt.p, (int64_t *)P.tc_ptr.p, nb));
        HIPCHK(hipMemcpyAsync(P.tc_fill.p, P.tc_ptr.p, sizeof(int64_t) * nb,
                              hipMemcpyDeviceToDevice, st));
        HIPCHK(bsr_colfill(nb, (const int32_t *)T.lo.p, (const int64_t *)T.woff.p,
                           (const uint2 *)T.rt.p, (const int64_t *)T.tb.p, (int64_t *)P.tc_fill.p,
                           uk, ut, st));
        HIPCHK(bsr_colsort((const int64_t *)P.tc_ptr.p, nb, uk, ut, sk, stt, st));
        cptr = (const int64_t *)P.tc_ptr.p;
        ck = sk;
        ct = stt;
    }
    // work items: four output tiles of one block row of T each
    CHK(ensure(P, P.g_cnt, sizeof(int64_t) * (nb + 1)));
    CHK(ensure(P, P.g_ofs, sizeof(int64_t) * (nb + 1)));
    HIPCHK(bsr_groups4((const int64_t *)T.tb.p, nb, (int64_t *)P.g_cnt.p, st));
    CHK(scan(P, (const int64_t *)P.g_cnt.p, (int64_t *)P.g_ofs.p, nb));
    // launched on a bound of the work-item count (each block row rounds up
    // once); the kernel reads the exact count, g_ofs[nb]
    const int64_t nwork = T.ntiles / 4 + nb + 1;
    CHK(ensure(P, P.g_owner, sizeof(int32_t) * (nwork + 1)));
    HIPCHK(work_owner((const int64_t *)P.g_ofs.p, nb, (int32_t *)P.g_owner.p, st));
    CHK(ensure(P, P.adj_tiles, sizeof(double) * 256 * (size_t)(T.ntiles + 1)));
    CHK(ensure(P, P.adj_tilesA, sizeof(double) * 256 * (size_t)(T.ntiles + 1)));
    const bool prof = P.opts.profile == 1 && P.have_events;
    if (prof) HIPCHK(hipEventRecord(P.ev[4], st));
    if (light_profile(P)) CHK(ktimer_mark(P, 1));
    HIPCHK(bsr_adjoint(nb, (const int32_t *)T.lo.p, (const int64_t *)T.woff.p,
                       (const uint2 *)T.rt.p, (const int64_t *)T.tb.p,
                       (const int32_t *)T.cols.p, (const double *)T.tA.p,
                       (const double *)T.tB.p, (const int32_t *)G.lo.p,
                       (const int64_t *)G.woff.p, (const uint2 *)G.rt.p,
                       (const int64_t *)G.tb.p, (const int32_t *)G.cols.p, (const double *)G.tA.p,
                       (const double *)G.tB.p, cptr, ck, ct,
                       (const int64_t *)P.g_ofs.p, (const int32_t *)P.g_owner.p,
                       (double *)P.adj_tiles.p,
                       (double *)P.adj_tilesA.p, (const int64_t *)P.g_ofs.p + nb, nwork, st,
                       T.b_only));
    if (light_profile(P)) CHK(ktimer_mark(P, 1));
    if (prof) {
        HIPCHK(hipEventRecord(P.ev[5], st));
        HIPCHK(hipEventSynchronize(P.ev[5]));
        float t;
        HIPCHK(hipEventElapsedTime(&t, P.ev[4], P.ev[5]));
        P.stats.adj_tile_launches += 1;
        P.stats.adj_tile_ms += t;
        // algorithmic work of the step: the partial products of G T^T and
        // T^T G that land in T's pattern, counted by the masked row product
        // on all-ones values (exact integers in double), 2 flops each, plus
        // 2 per mask entry; bytes: G and T read once, the output written
        double pp = 0.0;
        CHK(count_adjoint_products(P, Tp, Tk, &pp));
        P.stats.adj_tile_flops += 2.0 * pp + 2.0 * (double)Tp.nnz;
        P.stats.adj_tile_bytes += 12.0 * (double)Tk.nnz + 20.0 * (double)Tp.nnz;
    }
    if (want_csr) CHK(gather_tiles(P, Tp, T, (const double *)P.adj_tiles.p, out));
    return EXPM_OK;
}

bool light_profile(const expm_plan_s &P) { return P.opts.profile == 2 && P.have_events; }

int ktimer_mark(expm_plan_s &P, int kind) {
    if (P.kt_used == P.kt_ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        P.kt_ev.push_back(e);
    }
    HIPCHK(hipEventRecord(P.kt_ev[P.kt_used], P.st));
    if (P.kt_used % 2 == 0) P.kt_kind.push_back((char)kind);
    ++P.kt_used;
    return EXPM_OK;
}

void ktimer_collect_set(expm_plan_s &P, std::vector<hipEvent_t> &ev, std::vector<char> &kind,
                       size_t &used) {
    for (size_t j = 0; j + 1 < used; j += 2) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[j], ev[j + 1]) != hipSuccess) continue;
        if (kind[j / 2] == 0) {
            P.stats.tile_launches += 1;
            P.stats.tile_ms += t;
        } else {
            P.stats.adj_tile_launches += 1;
            P.stats.adj_tile_ms += t;
        }
    }
    (void)hipGetLastError();
    used = 0;
    kind.clear();
}

void ktimer_collect(expm_plan_s &P) { ktimer_collect_set(P, P.kt_ev, P.kt_kind, P.kt_used); }

// The timers of a forward run in profile mode 2, once its events are done.
void collect_forward(expm_plan_s &P) {
    if (!P.fwd_pending) return;
    (void)hipEventSynchronize(P.ev[7]);
    float t = 0.f;
    if (hipEventElapsedTime(&t, P.ev[6], P.ev[7]) == hipSuccess) P.stats.t_total_ms = t;
    ktimer_collect_set(P, P.kt_ev_fwd, P.kt_kind_fwd, P.kt_used_fwd);
    P.fwd_pending = false;
}

int gather_tiles(expm_plan_s &P, const DCsr &A, const TileSet &ts, const double *tiles,
                 double *out) {
    HIPCHK(bsr_gather(A.view(), (const int32_t *)ts.lo.p, (const int64_t *)ts.woff.p,
                      (const uint2 *)ts.rt.p, (const int64_t *)ts.tb.p, tiles, out, P.st));
    return EXPM_OK;
}

}  // namespace host
}  // namespace xpm
