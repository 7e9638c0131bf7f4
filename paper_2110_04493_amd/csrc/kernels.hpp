// Launch wrappers of the gfx950 kernels.  Every wrapper enqueues on `st` and
// returns the status of the launch (hipSuccess or the launch error).
#pragma once

#include "common.hpp"

namespace xpm {

// Number of row classes of the bitmap and accumulator kernels (the last one
// keeps its working set in global memory).
constexpr int kSymClasses = 5;
constexpr int kNumClasses = 9;

// Per-wave LDS capacity (bytes) of each class; the last class is global.
extern const int kSymCap[kSymClasses];
extern const int kNumCap[kNumClasses];

// Filter controller of Algorithm 4.1, resident in device memory.
struct FilterCtl {
    double eg;      // budget eps_g
    double er;      // tolerance e_r
    double theta;   // current entry threshold eps_f
    double b;       // norm of the current drop set
    double m;       // m_n
    int iter, maxit, done, status;
    unsigned arrive;  // blocks finished in the current pass
};

// ------------------------------------------------------------- scan
// out[0] = 0, out[i+1] = out[i] + in[i] for i < n; int64 counts.
hipError_t scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes,
                    hipStream_t st);
size_t scan_tmp_bytes(int64_t n);

// ------------------------------------------------------------- checks, norms
// flag |= 1: rowptr not monotone / bad start; 2: column out of range or not
// increasing; 4: non-finite value.
hipError_t validate_csr(CsrView A, int64_t nnz, int *flag, hipStream_t st);
// part[b] partial sums of v^2 over fixed chunks, then a fixed-order sum into *out.
hipError_t sumsq(const double *v, const int64_t *count, int64_t maxcount, double *part, int nparts,
                 double *out, hipStream_t st);
hipError_t scale_ldexp(const double *in, double *out, int64_t m, int e, hipStream_t st);
hipError_t negate_values(double *v, int64_t m, hipStream_t st);
// *out = sum of v[0..m) in a fixed order (block partials, then one block).
hipError_t sum_values(const double *v, int64_t m, double *part, int nparts, double *out,
                      hipStream_t st);
// out = ldexp(a + b, e), elementwise.
hipError_t add_scaled_ldexp(const double *a, const double *b, double *out, int64_t m, int e,
                            hipStream_t st);
// flags[0] = 1 if pattern(A) == pattern(B); flags[1] = values equal; flags[2] = values negated.
hipError_t compare_csr(CsrView A, CsrView B, int64_t nnz, int *flags, hipStream_t st);

// ------------------------------------------------------------- SpGEMM
// Row bounds of C = A*B (+ alphaA*A if addA): bitmap origin lo (multiple of
// 32), bitmap words, and the number of partial products ub.
hipError_t row_bounds(CsrView A, CsrView B, int addA, int32_t *lo, int64_t *words, int64_t *ub,
                      hipStream_t st);
// Class of every row from a per-row byte requirement (kind 0 symbolic, 1
// numeric, 2 complex numeric); rows listed per class.
// counts[kClasses] must be zeroed by the caller (done inside); lists is
// kClasses * n int32.
hipError_t bin_rows(const int64_t *words, const int64_t *cnt, int64_t n, int kind, int *counts,
                    int32_t *lists, hipStream_t st);
// Structural row counts of C and the column bitmaps of every row.
hipError_t symbolic(CsrView A, CsrView B, int addA, const int32_t *lo, const int64_t *woff,
                    uint32_t *bitmaps, int64_t *cnt, const int *host_counts, const int32_t *lists,
                    int64_t n, hipStream_t st);
// Numeric values: C = alphaA*A + A*B, then divided by `div` (1 = none).
// Rows sorted by column.  rowsq (optional): per-row sum of (c_ij + delta_ij)^2
// plus 1 when row i stores no diagonal entry.
hipError_t numeric(CsrView A, CsrView B, double alphaA, double div, const int32_t *lo,
                   const int64_t *woff, const uint32_t *bitmaps, const int64_t *crp, int32_t *cci,
                   double *cv, double *rowsq, const int *host_counts, const int32_t *lists,
                   int64_t n, void *scratch, const int64_t *scratch_off, hipStream_t st);
// The same product on complex values: A.v, B.v and cv hold a (real,
// imaginary) pair of doubles per entry; alphaA and div are real; rowsq as
// above with |c_ij + delta_ij|^2.  Rows binned with kind 2.
hipError_t numeric_z(CsrView A, CsrView B, double alphaA, double div, const int32_t *lo,
                     const int64_t *woff, const uint32_t *bitmaps, const int64_t *crp,
                     int32_t *cci, double *cv, double *rowsq, const int *host_counts,
                     const int32_t *lists, int64_t n, void *scratch, const int64_t *scratch_off,
                     hipStream_t st);
// Per-row byte requirement of the global-memory numeric class (for scratch;
// cplx: the complex accumulators).
hipError_t numeric_scratch_sizes(const int64_t *woff, const int64_t *crp, int64_t n,
                                 int64_t *bytes, hipStream_t st, bool cplx = false);

// ------------------------------------------------------------- filter
hipError_t filter_init(FilterCtl *c, double eg_scale, const double *norm2, double er, int maxit,
                       hipStream_t st);
hipError_t filter_init_theta(FilterCtl *c, double theta, hipStream_t st);
// One Algorithm 4.1 pass (sum of v^2 over |v| <= theta) plus the controller
// update; no-ops once the controller is done.
// The same pass over candidate tiles of 256 values.  tmin[t] / tmax[t] are
// the smallest nonzero and the largest magnitude of tile t and tsq[t] its
// sum of squares: a tile whose nonzeros all exceed the current threshold is
// skipped, one whose slots are all at most the threshold adds tsq[t], and
// only the tiles in between are read.  krc (may be NULL) receives, for
// every tile the pass reads, its entries above the pass's threshold per tile
// row (the trc layout of the product); since a tile is read exactly when
// its smallest nonzero is at most the threshold and its largest magnitude
// above it, the last pass leaves the final counts of every such tile.
// tmir (may be NULL): for a symmetric candidate formed on and right of the
// diagonal, per tile the index of its mirror tile (its transpose, left of
// the diagonal), -1 for a diagonal tile and -2 for a mirror: mirrors are
// not read, their partners count twice, and krc of each mirror receives
// its partner's column counts.
hipError_t filter_pass_tiles(const double *tiles, const double *tmin, const double *tmax,
                             const double *tsq, int64_t ntiles, FilterCtl *c, double *part,
                             int nparts, uint4 *krc, hipStream_t st,
                             const int64_t *tmir = nullptr);
hipError_t filter_pass(const double *v, const int64_t *count, int64_t maxcount, FilterCtl *c,
                       double *part, int nparts, hipStream_t st);
// Kept counts per row (|v| > theta); with addI the identity is added (E = I + T).
// With row_inst, row i uses controller c[row_inst[i]] and (if inst_addI is
// given) inst_addI[row_inst[i]] in place of addI.
hipError_t count_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                      const FilterCtl *c, int addI, int64_t *cnt, hipStream_t st,
                      const int32_t *row_inst = nullptr, const int *inst_addI = nullptr);
hipError_t write_kept(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                      const FilterCtl *c, int addI, const int64_t *orp, int32_t *oci, double *ov,
                      hipStream_t st, const int32_t *row_inst = nullptr,
                      const int *inst_addI = nullptr);

// ------------------------------------------------------------- 16 x 16 tiles
// (see bsr.hip).  nb = ceil(n / 16) block rows.
size_t bsr_lds_words(int64_t n);
hipError_t bsr_bounds(CsrView T, int64_t nb, int32_t *lo, int64_t *words, hipStream_t st);
hipError_t bsr_bitmap(CsrView T, int64_t nb, const int32_t *lo, const int64_t *woff, uint2 *rt,
                      int64_t *cnt, hipStream_t st);
hipError_t bsr_cbounds(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                       const int64_t *tb, int32_t *clo, int64_t *cwords, hipStream_t st);
hipError_t bsr_cpattern(int64_t n, int64_t nb, const int32_t *lo, const int64_t *woff,
                        const uint2 *rt, const int32_t *clo, const int64_t *cwoff, int64_t *ccnt,
                        const int64_t *ctb, int32_t *ccols, uint2 *crt, hipStream_t st);
// panels of 4 block rows sharing column groups (bsr.hip)
hipError_t bsr_panel_bounds(int64_t nb, const int32_t *clo, const int64_t *cwoff, int32_t *plo,
                            int64_t *pwords, hipStream_t st);
// upper: only block columns at or right of each panel's first block row
hipError_t bsr_panel_cols(int64_t n, int64_t nb, const int32_t *clo, const int64_t *cwoff,
                          const uint2 *crt, const int32_t *plo, const int64_t *pwoff,
                          int64_t *pcnt, const int64_t *pofs, int32_t *pcols, hipStream_t st,
                          bool upper = false);
int64_t bsr_panel_work_bound(int64_t ctiles, int64_t nb);
hipError_t bsr_panel_groups(const int64_t *pcnt, int64_t nb, int64_t *gcnt, hipStream_t st);
hipError_t bsr_tcols(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                     const int64_t *tb, int32_t *tcols, int32_t *trows, hipStream_t st);
hipError_t bsr_seg(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                   const int64_t *tb, int64_t *seg, hipStream_t st);
hipError_t bsr_assemble(CsrView T, int64_t ntiles, const int32_t *tcols, const int32_t *trows,
                        const int64_t *seg, double *tA, double *tB, hipStream_t st);
// Symmetric tile pattern: mir[t] = index of tile t's transpose (0 and
// *bad |= 1 where it is missing).
hipError_t bsr_tile_mirrors(int64_t ntiles, const int32_t *lo, const int64_t *woff,
                            const uint2 *rt, const int64_t *tb, const int32_t *tcols,
                            const int32_t *trows, int64_t *mir, int *bad, hipStream_t st);
// owner[w] = i for every w in [ofs[i], ofs[i + 1]), i < m (ofs: exclusive
// scan with the total in ofs[m]): the panel or block row of each work item
// of the tile product and adjoint kernels.
hipError_t work_owner(const int64_t *ofs, int64_t m, int32_t *owner, hipStream_t st);
// With upper (a symmetric C), the product forms the tiles on and right of
// the diagonal and writes each off-diagonal one's transpose (values and
// summaries) to the tile left of it; *bad |= 1 where that tile is missing;
// tmir (may be NULL) receives the pairing of filter_pass_tiles.  amir (may
// be NULL): T symmetric and assembled in the B layout only; its A operands
// are read from the B layout of each tile's transpose (amir[t]).
hipError_t bsr_numeric_panel(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                             const int64_t *tb, const int32_t *tcols, const double *tA,
                             const double *tB, const int64_t *pgofs, const int64_t *nwork_dev,
                             const int32_t *owner, const int64_t *pofs, const int32_t *pcols,
                             const int32_t *clo, const int64_t *cwoff, const uint2 *crt,
                             const int64_t *ctb, double *ctiles, int64_t n, double *tsq,
                             int32_t *tnz, double *tmn, double *tmx, uint4 *trc, double *bdg,
                             int64_t nwork, hipStream_t st, bool upper = false,
                             int *bad = nullptr, int64_t *tmir = nullptr,
                             const int64_t *amir = nullptr);
hipError_t bsr_norm_tiles(int64_t n, int64_t nb, const int64_t *ctb, const int64_t *ccnt,
                          const int32_t *ccols, const double *tsq, const int32_t *tnz,
                          const double *bdg, double *bsq, int64_t *bnz, hipStream_t st);
hipError_t bsr_rowsq(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, double *rowsq, hipStream_t st);
// Compaction of the candidate tiles (kept: |v| > c->theta) into CSR: kept
// counts per row, then the entries.  tmn / tmx / trc (may be NULL) are the
// per-tile summaries the product leaves with its norm partials; krc (may be
// NULL, only with tmn / tmx) holds the counts that the last pass of
// Algorithm 4.1 recorded for the tiles it read at the final threshold.
hipError_t bsr_count(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, const double *tmn, const double *tmx,
                     const uint4 *trc, const uint4 *krc, const FilterCtl *c, int64_t *cnt,
                     hipStream_t st, int32_t *rcnt = nullptr, const int64_t *rofs = nullptr);
hipError_t bsr_write(int64_t n, const int64_t *ctb, const int64_t *ccnt, const int32_t *ccols,
                     const double *ctiles, const double *tmx, const FilterCtl *c,
                     const int64_t *orp, int32_t *oci, double *ov, hipStream_t st);
// rounds of 64 tiles per block row (rnd[I] = ceil(ccnt[I] / 64)); the
// compaction with one wave per round (rofs: exclusive scan of rnd with the
// total at rofs[nb], owner its work map, rcnt the per-round row counts of
// bsr_count; nwork: a bound of the round count)
hipError_t bsr_rounds(const int64_t *ccnt, int64_t nb, int64_t *rnd, hipStream_t st);
hipError_t bsr_write_rounds(int64_t n, const int64_t *ctb, const int64_t *ccnt,
                            const int32_t *ccols, const double *ctiles, const double *tmx,
                            const FilterCtl *c, const int64_t *orp, const int32_t *rcnt,
                            const int64_t *rofs, const int32_t *owner, int64_t nwork,
                            int32_t *oci, double *ov, hipStream_t st);

// adjoint on tiles (bsr_adjoint.hip)
hipError_t bsr_colcount(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                        int64_t *cnt, hipStream_t st);
hipError_t bsr_colfill(int64_t nb, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                       const int64_t *tb, int64_t *fill, int32_t *uk, int64_t *ut,
                       hipStream_t st);
hipError_t bsr_colsort(const int64_t *ptr, int64_t nb, const int32_t *uk, const int64_t *ut,
                       int32_t *ck, int64_t *ct, hipStream_t st);
hipError_t bsr_groups4(const int64_t *tb, int64_t nb, int64_t *gcnt, hipStream_t st);
hipError_t bsr_adjoint(int64_t nb, const int32_t *tlo, const int64_t *twoff, const uint2 *trt,
                       const int64_t *ttb, const int32_t *tcols, const double *tA,
                       const double *tB, const int32_t *glo,
                       const int64_t *gwoff, const uint2 *grt, const int64_t *gtb,
                       const int32_t *gcols, const double *gA, const double *gB,
                       const int64_t *cptr, const int32_t *ck, const int64_t *ct,
                       const int64_t *gofs, const int32_t *owner, double *out, double *outA,
                       const int64_t *nwork_dev, int64_t nwork, hipStream_t st,
                       bool symT = false);   // symT: T symmetric, B layout only
hipError_t bsr_gather(CsrView T, const int32_t *lo, const int64_t *woff, const uint2 *rt,
                      const int64_t *tb, const double *tiles, double *out, hipStream_t st);

// ------------------------------------------------------------- batched
// Instance k of a block-diagonal stack owns rows [row_off[k], row_off[k+1]).
hipError_t fill_row_inst(const int64_t *row_off, int count, int64_t n, int32_t *row_inst,
                         hipStream_t st);
// Per-instance controller set-up: mode[k] 0 = search with budget
// eg_scale[k] * sqrt(norm2[k]) (norm2 may be NULL: budget eg_scale[k]),
// 1 = keep everything, 2 = drop everything.
hipError_t filter_init_batched(FilterCtl *c, int count, const double *eg_scale,
                               const double *norm2, const int *mode, double er, int maxit,
                               hipStream_t st);
// One Algorithm 4.1 pass for every instance whose controller is not done;
// instance k's candidate values are cv[crp[row_off[k]] .. crp[row_off[k+1]]).
hipError_t filter_pass_batched(const double *cv, const int64_t *crp, const int64_t *row_off,
                               int count, FilterCtl *c, double *part, int blocks_per_inst,
                               hipStream_t st);
// out[k] = sum of v over rows [row_off[k], row_off[k+1]) (fixed order).
hipError_t segment_sums(const double *v, const int64_t *row_off, int count, double *out,
                        hipStream_t st);
// out[k] = rp[row_off[k]] for k = 0..count.
hipError_t gather_offsets(const int64_t *rp, const int64_t *row_off, int count, int64_t *out,
                          hipStream_t st);
// Stacks instance CSRs (descriptor table on the device) into one
// block-diagonal CSR; values scaled by 2^-shift[k].
struct InstDesc {
    const int64_t *rp;
    const int32_t *ci;
    const double *v;
    int64_t n, row_off, nnz_off;
    int shift;
};
hipError_t stack_instances(const InstDesc *desc, int count, const int64_t *row_off, int64_t n,
                           int64_t *rp, int32_t *ci, double *v, hipStream_t st);
// Copies rows [r0, r0 + m) of a CSR into a standalone CSR with columns
// shifted by -r0.
hipError_t extract_block(const int64_t *rp, const int32_t *ci, const double *v, int64_t r0,
                         int64_t m, int64_t *orp, int32_t *oci, double *ov, hipStream_t st);

// ------------------------------------------------------------- sparse add
// C = A + B with exact zeros removed (two passes: count then write).
hipError_t add_count(CsrView A, CsrView B, int64_t *cnt, hipStream_t st);
hipError_t add_write(CsrView A, CsrView B, const int64_t *crp, int32_t *cci, double *cv,
                     hipStream_t st);
// T = S_1 + ... + S_m (m <= kSumMaxTerms terms of one n x n shape), summed
// entry by entry in term order (bitwise what adding the terms one after
// another gives) with exact zeros removed; two passes (count, then write).
// Rows whose column window or distinct-column bound exceeds the kernel's
// LDS slice work in global scratch: sum_terms_bounds gives each row's bytes
// (0 for LDS rows), and goff is their exclusive scan (n + 1 entries).
// *overflow is set if a row needed scratch it was not given.
constexpr int kSumMaxTerms = 32;
struct SumTerms {
    const int64_t *rp[kSumMaxTerms];
    const int32_t *ci[kSumMaxTerms];
    const double *v[kSumMaxTerms];
    int m;
};
hipError_t sum_terms_bounds(const SumTerms &T, int64_t n, int64_t *bytes, hipStream_t st);
hipError_t sum_terms_count(const SumTerms &T, int64_t n, char *gscr, const int64_t *goff,
                           int64_t *cnt, int *overflow, hipStream_t st);
hipError_t sum_terms_write(const SumTerms &T, int64_t n, char *gscr, const int64_t *goff,
                           const int64_t *orp, int32_t *oci, double *ov, hipStream_t st);
// out (aligned with T's entries) = the values of E = I + T (E as returned:
// exact zeros dropped, so E's row differs from T's at most at the diagonal)
// at T's entries; 0 where E dropped a diagonal entry.
hipError_t values_at_t(const int64_t *trp, const int32_t *tci, const int64_t *erp,
                       const double *ev, int64_t n, double *out, hipStream_t st);
// Identity matrix rows.
hipError_t fill_identity(int64_t n, int64_t *rp, int32_t *ci, double *v, hipStream_t st);

// ------------------------------------------------------------- transpose
// colcnt and fillpos: n int64 each; tmp_ci / tmp_v: nnz entries each (used
// for rows longer than the LDS sort).
hipError_t transpose(CsrView A, int64_t nnz, int64_t *trp, int32_t *tci, double *tv,
                     int64_t *colcnt, int64_t *fillpos, int32_t *tmp_ci, double *tmp_v,
                     void *scan_tmp, size_t scan_tmp_bytes, hipStream_t st);
// The transposed pattern with, in place of values, the position in A of
// every transposed entry (tpos / tmp_pos: nnz int64 each).
hipError_t transpose_index(CsrView A, int64_t nnz, int64_t *trp, int32_t *tci, int64_t *tpos,
                           int64_t *colcnt, int64_t *fillpos, int32_t *tmp_ci, int64_t *tmp_pos,
                           void *scan_tmp, size_t scan_tmp_bytes, hipStream_t st);

// ------------------------------------------------------------- masked products
// out[e] (aligned with the stored entries of mask M) =
//   gamma * D(i,j) + alpha1 * (A1*B1)(i,j) + alpha2 * (A2*B2)(i,j),
// for (i, j) in supp(M); D, A2/B2 optional (n == 0 views are skipped).
// The product terms are divided by `div` before being added.
struct MaskTerm {
    CsrView A, B;
    double alpha;
};
// Returns hipErrorOutOfMemory (with *needed set) when scratch is too small.
size_t masked_meta_bytes(int64_t n);
hipError_t masked_products(CsrView M, CsrView D, double gamma, MaskTerm t1, MaskTerm t2,
                           double div, double *out, void *scratch, size_t scratch_bytes,
                           size_t *needed, hipStream_t st);
// The same for one product whose left factor's rows and right factor's
// columns are both at hand, as inner products: for (r, c) in supp(M),
//   out[e] = (sum_k A(r,k) B(k,c)) / div + dv[e].
// A by rows: rp/ci of A, the value of entry p being av[apos[p]]; B by
// columns: rp/ci of B^T, the value of entry p being bv[bpos[p]].
struct PosCsr {
    const int64_t *rp;
    const int32_t *ci;
    const int64_t *pos;
    const double *v;
};
hipError_t masked_dot(CsrView M, const double *dv, PosCsr A, PosCsr Bt, double div, double *out,
                      hipStream_t st);

// ------------------------------------------------------------- complex values
// Value arrays hold a (real, imaginary) pair of doubles per entry (kernels.hip).
// Algorithm 4.1 on the moduli |z| = sqrt(re^2 + im^2).
hipError_t filter_pass_z(const double *v, const int64_t *count, int64_t maxcount, FilterCtl *c,
                         double *part, int nparts, hipStream_t st);
hipError_t count_kept_z(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                        const FilterCtl *c, int addI, int64_t *cnt, hipStream_t st);
hipError_t write_kept_z(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                        const FilterCtl *c, int addI, const int64_t *orp, int32_t *oci,
                        double *ov, hipStream_t st);
hipError_t add_count_z(CsrView A, CsrView B, int64_t *cnt, hipStream_t st);
hipError_t add_write_z(CsrView A, CsrView B, const int64_t *crp, int32_t *cci, double *cv,
                       hipStream_t st);
hipError_t compare_csr_z(CsrView A, CsrView B, int64_t nnz, int *flags, hipStream_t st);
hipError_t fill_identity_z(int64_t n, int64_t *rp, int32_t *ci, double *v, hipStream_t st);
// flag |= 4 if any of v[0..m) (doubles) is NaN or Inf.
hipError_t check_finite(const double *v, int64_t m, int *flag, hipStream_t st);
// dst[q] = conj(src[pos[q]]).
hipError_t gather_conj_z(const double *src, const int64_t *pos, int64_t m, double *dst,
                         hipStream_t st);

// ------------------------------------------------------------- symmetric iterates
// The entries right of the diagonal of T: row counts (orp == NULL) or the
// entries written at orp.  sym_rows: U + U^T from the transposed strictly
// upper part Lt and T's entries on and right of the diagonal (counts, or
// the entries at orp; rows in column order).
hipError_t triu_strict(CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci, double *ov,
                       hipStream_t st);
hipError_t sym_rows(CsrView Lt, CsrView T, int64_t *cnt, const int64_t *orp, int32_t *oci,
                    double *ov, hipStream_t st);

// ------------------------------------------------------------- extras.hip
hipError_t fill_f64(double *p, int64_t m, double x, hipStream_t st);
// *out = bit pattern of the largest row sum of |a_ij| (rows summed in order).
hipError_t row_abs_max(CsrView A, unsigned long long *out, hipStream_t st);
// The FPIM's fixed threshold on a candidate (CSR rows or tiles): the
// controller c is set to theta = eps * (largest column sum of |v|); colsum
// holds n doubles of workspace, mx one word.
hipError_t fpim_theta_rows(const int64_t *crp, const int32_t *cci, const double *cv, int64_t n,
                           double *colsum, unsigned long long *mx, double eps, FilterCtl *c,
                           hipStream_t st);
hipError_t fpim_theta_tiles(int64_t n, int64_t ntiles, const int32_t *ccols, const double *ctiles,
                            double *colsum, unsigned long long *mx, double eps, FilterCtl *c,
                            hipStream_t st);
// out[0] = l1, out[1] = l2 of Eq. (3.1) in the caller's ordering (order[]:
// library row -> caller row, or NULL); both LLONG_MIN for an empty matrix.
hipError_t band_of(CsrView T, const int32_t *order, long long *out, hipStream_t st);
// dst[q] = src[pos[q]]  /  dst[pos[q]] += src[q] (pos: a permutation).
hipError_t gather_pos(const double *src, const int64_t *pos, int64_t m, double *dst,
                      hipStream_t st);
hipError_t add_scatter_pos(const double *src, const int64_t *pos, int64_t m, double *dst,
                           hipStream_t st);
// Y = A X (X, Y dense row-major, leading dimensions ldx, ldy): from CSR, or
// from A's 16 x 16 tiles (A operand layout) on the matrix cores.
hipError_t spmm(CsrView A, int64_t m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                hipStream_t st);
hipError_t spmm_tiles(int64_t n, int64_t nb, const int64_t *tb, const int32_t *tcols,
                      const double *tA, int64_t m, const double *X, int64_t ldx, double *Y,
                      int64_t ldy, hipStream_t st);

}  // namespace xpm
