// Internal interface of the host executor shared by the single-matrix and
// batched drivers (not part of the C ABI).
#pragma once

#include <chrono>
#include <map>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/expm.h"
#include "kernels.hpp"

namespace xpm {
namespace host {

// ------------------------------------------------------------------ memory

// Grow-only device buffer from the stream-ordered pool.
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct DCsr {
    int64_t n = 0, nnz = 0;
    Buf rp, ci, v;
    CsrView view() const {
        return CsrView{n, (const int64_t *)rp.p, (const int32_t *)ci.p, (const double *)v.p};
    }
};

// A matrix held as 16 x 16 tiles: per block row the origin (block column,
// multiple of 32), bit-map words with prefix counts (rank table) and the
// base tile index; the tiles in the A and B operand layouts.
struct TileSet {
    Buf lo, words, woff, rt, cnt, tb, tA, tB, cols, rows, seg;   // cols / rows: block column
                                                                 // and row of every tile
    // for a symmetric matrix assembled in the B layout only: per tile the
    // index of its transpose, whose B-layout bytes are this tile's A layout
    Buf mir;
    int64_t nb = 0, ntiles = 0;
    bool b_only = false;
};


}  // namespace host
}  // namespace xpm

struct expm_plan_s {
    expm_opts opts{};
    hipStream_t st = nullptr;
    size_t live = 0, peak = 0;

    // Fixed-region mode (expm_sparse_noalloc): every workspace buffer is cut
    // from [arena, arena + arena_bytes) by a first-fit allocator over the
    // free ranges (offset -> length, adjacent ranges merged) instead of the
    // stream-ordered pool; everything runs on one stream, so a range freed
    // and handed out again is reused in stream order.  The output goes to
    // the caller's buffers na_rp / na_ci / na_v of na_cap entries (na_need:
    // nnz(E) once known).
    char *arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> arena_free;
    int64_t *na_rp = nullptr;
    int32_t *na_ci = nullptr;
    double *na_v = nullptr;
    int64_t na_cap = 0, na_need = -1;
    // the shadow plan a fixed-region call runs on (created with the plan)
    expm_plan_s *na = nullptr;

    // workspace
    xpm::host::Buf lo, words, woff, ub, cnt, crp, bitmaps, lists, counts, scan_tmp, part, ctl, rowsq, norm2,
        scratch, soff, sbytes, flags, krp, tmp1, tmp2;
    xpm::host::Buf cci, cv;            // candidate entries
    int *host = nullptr;    // pinned readback area
    // current matrices
    xpm::host::DCsr H0, S, Snew, T, Tnew, Hpat_t;
    // adjoint state
    bool have_fwd = false;
    int M = 0, N = 0, Mp = 0, ck = 1;
    double a = 0;
    std::vector<xpm::host::DCsr> taylor;        // S^_1 .. S^_M'
    std::vector<xpm::host::DCsr> ckpt;          // kept iterates T^_k, k = ckpt_at[j]
    // buffers of earlier calls' terms, checkpoints and recomputed iterates,
    // reused entry for entry so that repeated calls do not reallocate
    std::vector<xpm::host::DCsr> taylor_pool, ckpt_pool, seg_pool;
    std::vector<int> ckpt_at;                   // 0, then every ck back from N - 1
    xpm::host::DCsr TN;                         // T^_N
    // checkpoint j's iterate as tiles (pattern and both layouts), kept from
    // the forward product that took it as input, for that iterate's adjoint
    // step (T^_{N-1}, the largest, always when the last squaring ran on
    // tiles; the others within a memory budget)
    std::vector<xpm::host::TileSet> cts;
    std::vector<char> cts_ok;
    size_t dev_mem = 0;   // device memory in bytes (0: not queried yet)
    xpm::host::DCsr Epat;   // the returned E's size (its row pointers without reordering)
    std::vector<double> theta;       // squaring thresholds, 1..N
    bool zero_h = false;
    // stats / outputs
    expm_stats stats{};
    bool have_stats = false;
    std::vector<void *> outputs;
    // profiling: events around the phases of the last sparse product
    hipEvent_t ev[8] = {};
    bool have_events = false;
    // C's tile count and rank-table size, read back with T's tile count by
    // bsr_pattern(with_c) for the tile product that follows it
    bool c_pre = false;
    int64_t c_pre_tiles = 0, c_pre_words = 0;
    // opts.profile == 2: an event pair around every tile product (kind 0) and
    // adjoint tile (kind 1) launch, read once the call has synchronised
    std::vector<hipEvent_t> kt_ev;
    std::vector<char> kt_kind;
    size_t kt_used = 0;
    // ... and the forward's timers are read only after a later wait (the
    // end of expm_sparse_backward, expm_get_stats or the next forward), so
    // that expm_sparse returns without waiting: they move to this second
    // set, and ev[6] / ev[7] bracket the forward
    std::vector<hipEvent_t> kt_ev_fwd;
    std::vector<char> kt_kind_fwd;
    size_t kt_used_fwd = 0;
    bool fwd_pending = false;
    int64_t last_fma = 0;
    // 16 x 16 tile path of the squaring: T's tile pattern (origin, bit-map
    // words, rank tables, tile bases), its tiles in both operand layouts, C's
    // tile pattern, work items and the candidate tiles
    xpm::host::TileSet tsT, tsG;
    xpm::host::Buf c_lo, c_words, c_woff, c_cnt, c_tb, c_cols, c_tiles, g_cnt, g_ofs, b_sq, b_nz,
        c_rt;
    // per candidate tile: its share of ||I + T~||_F^2, its nonzero slots,
    // their smallest and largest magnitudes and the nonzeros of each row
    xpm::host::Buf c_sq, c_nz, c_mn, c_mx, c_rc, c_kc;
    // per block row: the diagonal tile's sum of (2 c_ii + 1)
    xpm::host::Buf b_dg;
    // panels of four block rows for the product (p_*: origin, words, column
    // counts and lists, work groups)
    xpm::host::Buf p_lo, p_words, p_woff, p_cnt, p_ofs, p_gcnt, p_gofs, p_cols, p_owner, g_owner;
    // block-column lists of T (the block rows of T^T) for the adjoint; the
    // adjoint step's output tiles in the B and A operand layouts
    xpm::host::Buf tc_cnt, tc_ptr, tc_fill, tc_k, tc_t, adj_tiles, adj_tilesA;
    std::vector<char> sq_path;       // per squaring step: 1 = tiles, 0 = scalar rows
    // locality reordering: order (new -> old), newidx (old -> new); H' = P H P^T
    // replaces H0 and E = P^T (I + T'_N) P; hmap gives, for each entry of H',
    // the index of the matching entry of H; tmap, for each entry of T'_N, the
    // index of the matching entry of the returned E (-1: none)
    bool perm_active = false;
    xpm::host::Buf order, newidx, hmap, tmap, ro_rb, ro_d0, ro_d1, ro_d3, ro_q0, ro_q1, ro_ell,
        ro_cell,
        ro_cnt, ro_off, ro_pcnt, ro_pw, ro_pofs, ro_gbits;
    xpm::host::DCsr Hp, Eperm;
    // tile fill of T from which the tile product is used (opts.tile_min_fill;
    // default 0.2, where the two paths cost about the same on MI355X at
    // n = 90,000 in natural order)
    double bsr_min_fill = 0.2;
    // EXPM_FILTER_FIXED_REL: the filter parameter eps of the running forward
    // (0 otherwise); column sums and a max word for its thresholds; the
    // bandwidth pairs (l1, l2) of T_0 .. T_N with opts.diagnostics
    double fpim_eps = 0.0;
    xpm::host::Buf colsum, amax, bands;
    int ordering = 0;   // the ordering applied by the running call: 0 none, 1 strips, 2 levels
    // H exactly symmetric (and opts.use_symmetry): T_0 is made exactly
    // symmetric and every squaring's tile product forms the candidate's
    // upper triangle only (the row product keeps exact symmetry by itself)
    bool sym_h = false;
    int last_sym = -1;   // exact symmetry found by the last normality test (-1: not run)
    xpm::host::Buf mirror_bad, sym_cnt;
    xpm::host::Buf c_mir;   // per candidate tile: its mirror, -1 (diagonal) or -2 (a mirror)
    // the compaction's rounds of 64 candidate tiles: per block row their
    // count and offsets, per round the kept entries of its 16 rows, work map
    xpm::host::Buf r_cnt, r_ofs, r_rows, r_owner;
};

namespace xpm {
namespace host {

constexpr int kParts = 1024;

// A named range for ROCm's tracing tools (rocprofv3 --marker-trace): the
// phases of a call show up on the timeline; without a tool attached the
// calls do nothing.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    // ends this range and opens the next phase's
    void next(const char *name) {
        roctxRangePop();
        roctxRangePushA(name);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Runs f when the enclosing scope ends: releases a function's local
// workspace on its error returns too (release is idempotent).
template <class F>
struct AtExit {
    F f;
    ~AtExit() { f(); }
};
template <class F>
AtExit<F> at_exit(F f) {
    return AtExit<F>{f};
}

extern thread_local std::string g_err;   // message of the calling thread's last error
double ms_since(std::chrono::steady_clock::time_point t0);
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int ensure(expm_plan_s &P, Buf &b, size_t bytes);
int reserve_as(expm_plan_s &P, Buf &b, const Buf &ref);
int reserve_as(expm_plan_s &P, DCsr &d, const DCsr &ref);
int reserve_as(expm_plan_s &P, TileSet &t, const TileSet &ref);
void release(expm_plan_s &P, Buf &b);
void release(expm_plan_s &P, DCsr &A);
// vw: doubles per value (2 for complex matrices)
int ensure_csr(expm_plan_s &P, DCsr &A, int64_t n, int64_t nnz, int vw = 1);
int copy_csr(expm_plan_s &P, DCsr &dst, const DCsr &src, int vw = 1);
// Appends an entry to live, reusing the buffers of the entry at the same
// position in an earlier call (kept in pool by retire).
DCsr &push_reuse(std::vector<DCsr> &live, std::vector<DCsr> &pool);
void retire(std::vector<DCsr> &live, std::vector<DCsr> &pool);
int sync(expm_plan_s &P);
int scan(expm_plan_s &P, const int64_t *in, int64_t *out, int64_t n);
void *out_alloc(expm_plan_s &P, size_t bytes);
void out_free(expm_plan_s &P, void *p);
// The three arrays of an output CSR with n rows and nnz entries: from the
// caller's allocator (or the pool), or, in fixed-region mode, the caller's
// buffers after a capacity check.  On failure nothing stays allocated.
int alloc_output(expm_plan_s &P, int64_t n, int64_t nnz, int64_t **rp, int32_t **ci,
                 double **v, int vw = 1);
double plan_r0(int M, double x);
int plan_mn(double nh, double eps, int *Mo, int *No);
// cplx: complex values (a (real, imaginary) pair of doubles per entry)
int spgemm(expm_plan_s &P, CsrView A, int64_t nnzA, CsrView B, double alphaA, double div,
           bool rowsq, int64_t *total, bool cplx = false);
int sparse_add(expm_plan_s &P, const DCsr &A, const DCsr &B, DCsr &dst);
int sum_taylor(expm_plan_s &P, DCsr &dst);
int transpose_csr(expm_plan_s &P, const DCsr &A, DCsr &dst);
int transpose_pos(expm_plan_s &P, const DCsr &A, DCsr &dst);
int detect_normal(expm_plan_s &P, const DCsr &H, double nh, int *normal);
int check_view(const expm_csr_cview *H);
// A fixed threshold already set in the filter controller on the device
// (theta_fixed argument of filter_and_count).
constexpr double kThetaOnDevice = -2.0;
int filter_and_count(expm_plan_s &P, int64_t n, int64_t cand, double eg_scale,
                     const double *norm2, bool use_fixed, double theta_fixed, bool addI,
                     FilterCtl *hctl, int64_t *kept, bool cplx = false);
int write_filtered(expm_plan_s &P, int64_t n, DCsr &dst, int64_t kept, bool addI,
                   bool exact_alloc, bool cplx = false);
int masked(expm_plan_s &P, CsrView M, CsrView D, double gamma, MaskTerm t1, MaskTerm t2,
           double div, double *out);
int plan_input(expm_plan_s &P, const expm_csr_cview *Hv, double eps, DCsr &dst,
               expm_analysis *A);
int forward(expm_plan_s &P, const expm_csr_cview *Hv, double eps, expm_csr *E);
// Algorithm 4.2 over C (complex.hip)
int forward_z(expm_plan_s &P, const expm_csr_cview *Hv, double eps, expm_csr *E);
// EXPM_LOG=1: one line of the call's statistics on stderr
void log_call(const expm_plan_s &P, int64_t n, double eps, int status);
void free_adjoint_state(expm_plan_s &P);
int bsr_pattern(expm_plan_s &P, CsrView T, int64_t nnz, TileSet &ts, double *fill,
                bool with_c = false);
// b_only: T is symmetric; only the B layout is assembled, with ts.mir
int bsr_tiles(expm_plan_s &P, CsrView T, TileSet &ts, bool b_only = false);
bool tiles_allowed(const expm_plan_s &P, int64_t n);
// upper: a symmetric candidate, formed on and right of the diagonal and
// mirrored to the left of it
int tile_product(expm_plan_s &P, CsrView T, bool prof, bool tile_norms, int64_t *ctiles_out,
                 bool upper = false);
int tile_candidates(expm_plan_s &P, CsrView T, int64_t *cand);
int square_step_bsr(expm_plan_s &P, const DCsr &T, DCsr &dst, double a_ri, bool use_fixed,
                    double theta_fixed, bool exact_alloc, int stat_i);
// One adjoint step on tiles: out (aligned with Tp's entries) =
// P_Tp(2 G + G Tp^T + Tp^T G), with G given on the pattern of Tk.  Tp's tile
// pattern must be in P.tsT (with t_tiles_ready also its tiles, else they
// are assembled here); with g_pattern_ready, P.tsG already holds Tk's,
// and with g_tiles_ready also G's values as tiles.  The output is left as
// tiles on Tp's pattern in P.adj_tiles / P.adj_tilesA, and written to out
// only with want_csr.
int adjoint_step_bsr(expm_plan_s &P, const DCsr &Tp, const DCsr &Tk, const double *g,
                     double *out, bool g_pattern_ready, bool g_tiles_ready, bool want_csr,
                     bool t_tiles_ready);
// Values of A's stored entries (CSR order) from tiles in the B layout on A's
// tile pattern ts.
int gather_tiles(expm_plan_s &P, const DCsr &A, const TileSet &ts, const double *tiles,
                 double *out);
void release(expm_plan_s &P, TileSet &ts);
// Kernel timers (opts.profile == 2): ktimer_mark records the next event of
// the pool on the plan's stream (call it before and after one launch);
// ktimer_collect, after the stream has synchronised, adds the measured pairs
// to the tile statistics and empties the pool.
bool light_profile(const expm_plan_s &P);
int ktimer_mark(expm_plan_s &P, int kind);
void ktimer_collect(expm_plan_s &P);
void collect_forward(expm_plan_s &P);
void ktimer_collect_set(expm_plan_s &P, std::vector<hipEvent_t> &ev, std::vector<char> &kind,
                       size_t &used);
int compute_reorder(expm_plan_s &P, CsrView G, int64_t nnz, int mode, bool *active);
// cplx: complex values (pairs of doubles)
int permute_csr(expm_plan_s &P, CsrView X, int64_t nnz, const int32_t *src_row,
                const int32_t *colmap, int64_t *orp, int32_t *oci, double *ov, int64_t *emap,
                bool cplx = false);
int permute_count(expm_plan_s &P, CsrView X, const int32_t *src_row, const int32_t *colmap,
                  int64_t *orp, bool ident, int64_t *total, int64_t *gwords);
int permute_write(expm_plan_s &P, CsrView X, int64_t nnz, const int32_t *src_row,
                  const int32_t *colmap, const int64_t *orp, int32_t *oci, double *ov,
                  int64_t *emap, int64_t *tmap, int64_t gwords, bool cplx, bool ident);
int scatter_map(expm_plan_s &P, const double *src, const int64_t *map, int64_t m, double *dst);
// dst[i] = src[map[i]], or 0 where map[i] < 0
int gather_map(expm_plan_s &P, const double *src, const int64_t *map, int64_t m, double *dst);

}  // namespace host
}  // namespace xpm

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            if (_e == hipErrorOutOfMemory)                                                 \
                return ::xpm::host::fail(EXPM_ENOMEM, "%s: out of device memory (%s:%d)",  \
                                         #expr, __FILE__, __LINE__);                       \
            return ::xpm::host::fail(EXPM_EHIP, "%s failed: %s (%s:%d)", #expr,            \
                                     hipGetErrorString(_e), __FILE__, __LINE__);           \
        }                                                                                  \
    } while (0)

#define CHK(expr)                     \
    do {                              \
        int _s = (expr);              \
        if (_s != EXPM_OK) return _s; \
    } while (0)
