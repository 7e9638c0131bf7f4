/*
 * expm.h - C ABI of the MI355X (gfx950) filtered precise-integration sparse
 * matrix exponential.
 *
 * Method: Wu, Zhang, Zhu, Hu, "High-performance computation of large sparse
 * matrix exponential" (arXiv 2110.04493), Algorithm 4.2.  Given a real sparse
 * H and a tolerance eps_tol, the library chooses the Taylor degree M and the
 * squaring count N from problem (4.20), builds the filtered Taylor seed
 * T_0 of e^{H 2^-N} - I (Eq. 4.10-4.14), runs the N filtered updates
 * T <- 2T + T*T of Eq. (2.7)/(4.15), each followed by the forward-error
 * filter of Algorithm 4.1, and returns E = I + T_N.  Every step runs in HIP
 * kernels on the GPU in IEEE double precision.
 *
 * Conventions shared by every entry point
 *  - Matrices are square CSR: rowptr int64[n+1], col int32[nnz] (sorted and
 *    unique within each row, 0 <= col < n), val double[nnz].  n < 2^31.
 *  - All matrix and gradient pointers are DEVICE pointers on the current HIP
 *    device.  Input views are borrowed: the library never writes or frees
 *    them and does not keep them after the call returns.
 *  - Every call is ordered on opts.stream (NULL = the null stream).  Calls
 *    block the host only where they must read a size or a scalar back from
 *    the device (allocation sizes, the norm of H, filter termination).
 *  - Return value: EXPM_OK (0) or a negative EXPM_E* code.  On error no
 *    output is allocated, the outputs are left zeroed, and expm_last_error()
 *    returns a message for the calling thread.
 *  - A plan is not thread-safe; separate plans may be used concurrently.
 *  - Outputs written on opts.stream are ready in stream order there only:
 *    expm_sparse returns without waiting for the device.
 *  - Tracing: each call marks its phases (plan, Taylor seed, squarings,
 *    finish; adjoint squarings and seed) as ROCTX ranges; with EXPM_LOG=1
 *    in the environment every expm_sparse call prints one line of its
 *    statistics on stderr.
 */
#ifndef EXPM_H
#define EXPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXPM_OK 0
#define EXPM_EINVAL (-1)   /* malformed CSR, NaN/Inf values, eps out of range     */
#define EXPM_ENOMEM (-2)   /* device allocation failed                            */
#define EXPM_EHIP (-3)     /* a HIP runtime call failed                           */
#define EXPM_ERANGE (-4)   /* no (M, N) with M <= 170 satisfies problem (4.20)    */
#define EXPM_ENOTCONV (-5) /* Algorithm 4.1 hit opts.max_filter_iter             */
#define EXPM_ENOTIMPL (-6) /* option combination not provided                    */
#define EXPM_ESTATE (-7)   /* call out of order (e.g. backward without forward)   */

#define EXPM_NORMAL_AUTO (-1)
#define EXPM_FILTER_PAPER 0 /* Algorithm 4.1 with the budgets of Algorithm 4.2    */
#define EXPM_FILTER_NONE 1  /* a = 0: plain precise integration, only exact zeros
                               are dropped (section 4.2: a_i = 0 is the original
                               method)                                            */
#define EXPM_FILTER_FIXED_REL 2 /* the FPIM's fixed filter (section 2): the Taylor
                               terms keep every nonzero (a = 0); T_0 and each
                               squaring candidate lose their entries with
                               |v| <= eps ||.||_1 (largest absolute column sum
                               of that matrix); eps is then the filter
                               parameter, and still sets (M, N) by (4.20)     */

#define EXPM_NORM_FRO 0     /* ||H|| of Algorithm 4.2 steps 1-3: Frobenius       */
#define EXPM_NORM_ONE 1     /* ... or the 1-norm (largest absolute column sum)    */

#define EXPM_MAXSTEP 128

/* Borrowed read-only CSR view: device pointers, or host pointers when
 * on_host = 1 (expm_sparse, expm_sparse_noalloc, expm_analyze,
 * expm_power_norms and expm_spmm's matrix then copy it to the device
 * first; expm_sparse_batched takes device views only). */
typedef struct {
    int64_t n, nnz;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
    int on_host;
} expm_csr_cview;

/* Output CSR (device pointers).  Owned by the caller's allocator when one is
 * given in expm_opts, else by the library; release with expm_csr_release()
 * or expm_free(). */
typedef struct {
    int64_t n, nnz;
    int64_t *rowptr;
    int32_t *col;
    double *val;
} expm_csr;

/* Optional device allocator for outputs.  alloc returns a device pointer of
 * at least `bytes` bytes usable on `stream` (NULL on failure); free releases
 * one.  Workspace is always allocated by the library itself. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} expm_allocator;

typedef struct {
    int normal;              /* Algorithm 4.2 step 2: -1 detect (exact symmetric
                                or skew-symmetric, else ||HH^T - H^TH||_F <=
                                16 u ||H||_F^2), 0 non-normal, 1 normal        */
    int filter_mode;         /* EXPM_FILTER_PAPER (default) | EXPM_FILTER_NONE */
    double e_r;              /* Algorithm 4.1 tolerance e_r (default 0.1)      */
    int max_filter_iter;     /* Algorithm 4.1 iteration cap (default 64)       */
    int keep_checkpoints;    /* 1: keep what expm_sparse_backward needs         */
    int checkpoint_interval; /* squaring iterates the adjoint keeps: c >= 1
                                keeps every c-th one counted back from T_{N-1}
                                (1 keeps all of them); -1 keeps ceil(sqrt(N))
                                of them, the last iterates T_{N-C} .. T_{N-1},
                                the costliest to recompute; 0 (default) keeps
                                those and also the earlier iterates, one
                                after another, while their CSR arrays fit in
                                a sixteenth of the device memory (then the
                                adjoint recomputes nothing)                  */
    void *stream;            /* hipStream_t for every launch and copy          */
    const expm_allocator *allocator; /* outputs; NULL = library allocation     */
    int profile;             /* 1: time the kernel phases of every squaring
                                step with HIP events on `stream` and count
                                the algorithmic work (fields t_*, sq_fma,
                                sq_in, tile_* and adj_tile_* of expm_stats);
                                this waits for the device after every step.
                                2: only an event pair around every launch of
                                the tile product and the adjoint tile kernel
                                (fields tile_launches, tile_ms,
                                adj_tile_launches, adj_tile_ms; tile_flops
                                stays 0), and one around the whole forward
                                (t_total_ms); expm_sparse does not wait for
                                them: they are read at the next wait of the
                                plan (the end of expm_sparse_backward,
                                expm_get_stats, or the next call).
                                0 (default): off                              */
    int reorder;             /* locality reordering: the rows and columns of H
                                are permuted symmetrically (strips of graph
                                distances) before the method runs and E is
                                permuted back, so that band tiles of the late
                                squarings are fuller.  Results are those of
                                the unpermuted method up to rounding order.
                                -1 (default) on for n >= 4096 when the tile
                                product can run, 0 off, 1 on; where the
                                graph has no 2D structure (path-like, or
                                small diameter) the level ordering below is
                                taken instead when it narrows the band.
                                2: the level ordering (Cuthill-McKee-like:
                                breadth-first levels from a far node, then
                                the distance from a second far node)         */
    double tile_min_fill;    /* a squaring step (and its adjoint) runs on 16x16
                                tiles when T's stored entries fill at least
                                this fraction of its tiles: < 0 (default)
                                picks 0.2, 0 always tiles, > 1 never          */
    int norm;                /* EXPM_NORM_FRO (default) | EXPM_NORM_ONE: the
                                norm of H in problem (4.20), in a and in the
                                Taylor budget (Algorithm 4.2 steps 1-3); the
                                normality test, Algorithm 4.1 and the
                                squaring budgets stay in the Frobenius norm  */
    int exact_ri;            /* 0 (default): r_i = 2^i r0, the paper's
                                simplification; 1: r_i = 2 r_{i-1} + r_{i-1}^2,
                                the recurrence of Eq. (4.3)                   */
    int diagnostics;         /* 1: per-step bandwidths l(T^_i) of Eq. (3.1),
                                in the caller's ordering, into expm_stats
                                (one extra pass over every iterate)          */
    int literal_a;           /* filter constant a for non-normal H:
                                0 (default) min(1/(N+1), 1/||H||); 1 the
                                1/||H|| of Algorithm 4.2 step 2 and section
                                4.2, also where it exceeds 1/(N+1)           */
    int batch_solo_n;        /* expm_sparse_batched: instances of order n >=
                                this run one after another through the
                                single-matrix path (locality ordering, tiles
                                sized to the instance); the others share the
                                stacked pass.  Default 4096; 0 stacks every
                                instance                                     */
    int use_symmetry;        /* 1 (default): for an exactly symmetric H (every
                                T_i is then symmetric) the summed Taylor seed
                                is made exactly symmetric (its upper triangle
                                mirrored; the terms agree to rounding) and
                                each tile product forms the candidate's tiles
                                on and right of the diagonal only, the others
                                being their transposes; 0: every tile formed */
} expm_opts;

/* Per-call statistics (indices as in the paper: Taylor term i = 2..M',
 * squaring step i = 1..N). */
typedef struct {
    int status, M, N, taylor_terms, normal, squarings;
    double a, norm_h, h0, r0, eg0;
    double taylor_theta[EXPM_MAXSTEP];
    int taylor_iters[EXPM_MAXSTEP];
    int64_t taylor_cand[EXPM_MAXSTEP], taylor_kept[EXPM_MAXSTEP];
    double sq_theta[EXPM_MAXSTEP], sq_normF[EXPM_MAXSTEP], sq_budget[EXPM_MAXSTEP];
    double sq_dropped[EXPM_MAXSTEP];
    int sq_iters[EXPM_MAXSTEP];
    int64_t sq_cand[EXPM_MAXSTEP], sq_kept[EXPM_MAXSTEP];
    int64_t nnz_e;
    size_t peak_workspace_bytes;
    /* with opts.profile == 1: per squaring step i, the partial products of
     * T*T (sq_fma), the stored entries of the input iterate (sq_in), and the
     * device time in ms of the symbolic, numeric and filter+compaction
     * phases; t_taylor_ms is the whole Taylor phase.  t_total_ms is the
     * last expm_sparse call: its wall time after a final wait with profile
     * 1, its device time between two events with profile 2, and only the
     * host's part of it with profile 0 (no final wait).  t_backward_ms is
     * the wall time of the last expm_sparse_backward call, which always
     * ends with a wait. */
    int64_t sq_fma[EXPM_MAXSTEP], sq_in[EXPM_MAXSTEP];
    double t_sym_ms[EXPM_MAXSTEP], t_num_ms[EXPM_MAXSTEP], t_filter_ms[EXPM_MAXSTEP];
    double t_taylor_ms, t_backward_ms, t_total_ms;
    /* with opts.profile 1 or 2, summed over every launch of the 16x16 tile
     * squaring product since the last expm_sparse began (its forward steps,
     * then the recomputation inside expm_sparse_backward): launches, device
     * time in ms (events on the plan's stream around each launch), and, with
     * profile 1 only, algorithmic flops, 2 per partial product of T*T plus 2
     * per stored entry of T (the 2T term), zero padding of the tiles not
     * counted.  adj_tile_* covers the tile kernel of the adjoint step the
     * same way (time only). */
    int64_t tile_launches;
    double tile_ms, tile_flops;
    int64_t adj_tile_launches;
    double adj_tile_ms;
    /* per squaring step: the number of 16x16 candidate tiles its product
       filled (capped at INT32_MAX), or 0 when it ran on scalar rows */
    int sq_tiles[EXPM_MAXSTEP];
    /* the error bound r_i of step i (2^i r0, or Eq. (4.3) with exact_ri) */
    double sq_ri[EXPM_MAXSTEP];
    /* with opts.diagnostics: l(T^_i) of Eq. (3.1) for i = 0..N, in the
       caller's row and column order (-1 when not computed) */
    int64_t sq_band[EXPM_MAXSTEP];
    /* EXPM_FILTER_FIXED_REL: the threshold T_0 was filtered with */
    double theta0;
    /* with opts.profile == 1, over the same launches as tile_flops: the
       algorithmic bytes of the tile product (12 per stored entry of T read
       once, 8 (n + 1) for its row pointer, 12 per nonzero candidate written
       once; for a symmetric T, whose product forms the partial products on
       and right of the diagonal only, tile_flops counts those), and the
       algorithmic flops and bytes of the adjoint tile step:
       2 per partial product of G T^T and T^T G that lands in the mask plus
       2 per mask entry; 12 per stored entry of G and of T read once, 8 per
       mask entry written */
    double tile_bytes, adj_tile_flops, adj_tile_bytes;
    /* the locality ordering applied: 0 none, 1 strips, 2 levels */
    int ordering;
    /* 1 when the last expm_sparse_backward ran its first step on the rows
       of the nonzeros of dL/dE (fewer than a hundredth of E's entries) */
    int adj_sparse_first;
    /* 1 when H was exactly symmetric and opts.use_symmetry formed only the
       upper triangle of each tile candidate */
    int symmetric;
} expm_stats;

typedef struct expm_plan_s *expm_plan_t;

/* Fills opts with the defaults listed above. */
void expm_opts_default(expm_opts *opts);

/* Creates a plan: the stream, options and the device workspace pool that
 * every later call on it reuses.  opts may be NULL (defaults).  Errors:
 * EXPM_EINVAL (bad option values), EXPM_EHIP. */
int expm_plan(expm_plan_t *out, const expm_opts *opts);

/* Algorithm 4.2: E ~= e^H.  H is a borrowed device CSR view; eps = eps_tol,
 * the relative error tolerance of problem (4.20), with 2^-60 <= eps < 1
 * (tolerances down to the unit roundoff of section 4.4 and slightly below,
 * as in section 5.2, are accepted).  *E receives a newly allocated device
 * CSR with sorted columns and no explicit zeros.  When the plan keeps
 * checkpoints, the state needed by expm_sparse_backward replaces that of the
 * previous call.  Errors: EXPM_EINVAL, EXPM_ERANGE, EXPM_ENOTCONV,
 * EXPM_ENOMEM, EXPM_EHIP. */
int expm_sparse(expm_plan_t p, const expm_csr_cview *H, double eps, expm_csr *E);

/* Algorithm 4.2 for a complex H: the paper states the method for H in
 * C^{n x n} (section 4).  H->val points at 2 nnz doubles, the real and the
 * imaginary part of each entry in turn (the layout of C99 double _Complex
 * and std::complex<double>), and E->val receives 2 nnz(E) doubles the same
 * way.  The steps are those of expm_sparse with complex arithmetic: the
 * normality test of step 2 compares H H^* with H^* H (an exactly Hermitian
 * or skew-Hermitian H is normal), and Algorithm 4.1 filters by the modulus
 * |z| = sqrt(re^2 + im^2), summing |z|^2 over the dropped entries.  Every
 * product runs on scalar rows (no tile path); the locality reordering runs
 * only when opts.reorder >= 1 (the default, -1, leaves complex H in its
 * order: the row products gain nothing from it).
 * Options as for expm_sparse, except: filter_mode EXPM_FILTER_FIXED_REL and
 * norm EXPM_NORM_ONE give EXPM_ENOTIMPL, and no adjoint is kept (a later
 * expm_sparse_backward returns EXPM_ESTATE).  Statistics as for expm_sparse.
 * Errors: those of expm_sparse, EXPM_ENOTIMPL. */
int expm_sparse_z(expm_plan_t p, const expm_csr_cview *H, double eps, expm_csr *E);

/* Adjoint of the last expm_sparse call on p (which must have run with
 * keep_checkpoints = 1): given dL/dE aligned with the stored entries of that
 * E (device double[nnz(E)]), writes dL/dH aligned with the stored entries of
 * its H (device double[nnz(H)], caller-allocated).  It is the exact
 * derivative of the map Algorithm 4.2 evaluates with every filter mask and
 * threshold held fixed: for the squarings of Eq. (4.15),
 * G_{k-1} = P_{k-1}(2 G_k + G_k T_{k-1}^T + T_{k-1}^T G_k), then the Taylor
 * recursion of Eq. (4.11) and the 2^-N scaling.  Squaring iterates between
 * checkpoints are recomputed.  Errors: EXPM_ESTATE, EXPM_ENOMEM, EXPM_EHIP. */
int expm_sparse_backward(expm_plan_t p, const double *dE_vals, double *dH_vals);

/* Algorithm 4.2 for `count` independent matrices H[k] with tolerances
 * eps[k] (host array), in one pass: every kernel launch of a step serves
 * the rows of all instances still active at that step.  Instances of order
 * at least opts.batch_solo_n run after that pass, one by one, as
 * expm_sparse would run them.  E[k] as for expm_sparse.  Errors as
 * expm_sparse; on error no E[k] is allocated. */
int expm_sparse_batched(expm_plan_t p, int count, const expm_csr_cview *H, const double *eps,
                        expm_csr *E);

/* Statistics of the last expm_sparse call (for batched calls, of the last
 * instance).  Errors: EXPM_ESTATE if no call has run. */
int expm_get_stats(expm_plan_t p, expm_stats *out);

/* The plan of Algorithm 4.2 for one input, before running it. */
typedef struct {
    int64_t n, nnz;
    double norm_h;     /* ||H|| in opts.norm                                  */
    double norm_fro;   /* ||H||_F (the normality test's scale)                */
    int M, N;          /* problem (4.20) at norm_h and eps                    */
    int normal;        /* Algorithm 4.2 step 2 (test or opts.normal)          */
    double a;          /* filter constant: 1/(N+1), or min(1/(N+1), 1/||H||)
                          for non-normal H (1/||H|| with opts.literal_a); 0
                          without the paper's filter                          */
    double h0, r0;     /* ||H 2^-N|| and the bound of Eq. (4.5)               */
    double eg0;        /* the Taylor terms' budget a r0 / (M e^{2 h0})        */
} expm_analysis;

/* Algorithm 4.2 steps 1-3 for H and eps_tol (as expm_sparse would take
 * them on this plan): validates H, computes its norms on the device, and
 * fills *out; nothing else runs and no output is allocated.  A zero H gives
 * M = N = 0.  Errors: EXPM_EINVAL, EXPM_ERANGE, EXPM_ENOMEM, EXPM_EHIP. */
int expm_analyze(expm_plan_t p, const expm_csr_cview *H, double eps, expm_analysis *out);

/* Y = A X on the device: A an n x n CSR view (typically E = e^H), X and Y
 * dense n x m, row-major with leading dimensions ldx, ldy >= m (device
 * pointers; Y must not overlap X).  Section 5.3 checks large exponentials
 * through E R with R = rand(n, 1000).  Each row of Y sums its products in
 * the column order of A's row.  Errors: EXPM_EINVAL, EXPM_ENOMEM, EXPM_EHIP. */
int expm_spmm(expm_plan_t p, const expm_csr_cview *A, int64_t m, const double *X, int64_t ldx,
              double *Y, int64_t ldy);

/* Time stepping with a computed exponential, Eq. (2.2): U_{k+1} = E U_k for
 * k = 0 .. steps-1, U_0 given (n x m, row-major, leading dimension m), and
 * U_steps written to U (device pointers; U may equal U0).  Errors as
 * expm_spmm. */
int expm_propagate(expm_plan_t p, const expm_csr_cview *E, int64_t m, const double *U0,
                   int steps, double *U);

/* ||H^k||_F for k = 1..K into out[0..K-1] (host array), by K - 1 unfiltered
 * sparse products on the device: the norms of the powers that h_{M,N} of
 * section 4.2 (the refinement before Eq. (4.9)) takes its maximum over.
 * Errors: EXPM_EINVAL, EXPM_ENOMEM, EXPM_EHIP. */
int expm_power_norms(expm_plan_t p, const expm_csr_cview *H, int K, double *out);

/* Host helper, Eq. (4.8)/(4.9): alpha-hat_i, the least M1 2^N1 (M1 >= 1,
 * 0 <= N1 <= 60) with 2^N1 r0(M1, x) <= r_i, where x = norm 2^(i-N-N1)
 * (Eq. 4.8, hk = NULL) or x = 2^(i-N-N1) max over M1+1 <= k <= 2M1+1 of
 * hk[k-1]^(1/k) with hk[k-1] = ||H^k|| for k = 1..K (Eq. 4.9, M1 then at
 * most (K-1)/2); for each N1 the least qualifying M1 is taken.
 * alpha-hat_i lambda(H) bounds the epsilon-bandwidth of e^{H 2^(i-N)}
 * (Eq. 4.7).  Errors: EXPM_EINVAL, EXPM_ERANGE (no pair qualifies). */
int expm_alpha_hat(double ri, int i, int N, double norm, const double *hk, int K,
                   int64_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as expm_sparse, with every device workspace buffer cut from a
 * static device array of EXPM_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each GPU it runs on until the process ends, and E written into
 * buffers the caller owns: E_rowptr int64[n+1], E_col int32[capacity],
 * E_val double[capacity] (device pointers; may be NULL when capacity is 0).
 * The call allocates and frees no device or pinned memory (host bookkeeping
 * uses the C++ heap); like expm_sparse it reads sizes back from the device.
 * Options come from the plan; keep_checkpoints and profile are ignored (no
 * expm_sparse_backward after this call: it returns EXPM_ESTATE).  Results
 * are ready in order on opts.stream.  Every call on one GPU shares that
 * GPU's array, whatever the plan: calls that overlap in time on one GPU
 * (other threads, other streams) race and must not be issued.
 * *nnz_e (may be NULL) receives nnz(E) once it is known, also when it
 * exceeds capacity.  Errors: those of expm_sparse, and EXPM_ENOMEM when the
 * workspace does not fit the static array (rejected up front when H alone
 * is too large) or nnz(E) > capacity. */
#define EXPM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int expm_sparse_noalloc(expm_plan_t p, const expm_csr_cview *H, double eps, int64_t *E_rowptr,
                        int32_t *E_col, double *E_val, int64_t capacity, int64_t *nnz_e);

/* Frees one output returned by this plan and zeroes *E. */
void expm_csr_release(expm_plan_t p, expm_csr *E);

/* Frees the plan, its workspace, checkpoints and unreleased outputs. */
void expm_free(expm_plan_t p);

/* Message describing the last error on the calling thread ("" if none). */
const char *expm_last_error(void);

/* Host helpers.  Eq. (4.5): r0(M, x) = (1/M!) sum_k x^{M+1+k}/(k!(M+1+k)),
 * the bound on ||F_0^{-1} R_0|| for degree M at ||H 2^-N|| = x. */
double expm_r0(int M, double x);

/* Problem (4.20): the (M, N) minimising M 2^N with ||H 2^-N|| <= 1 and
 * 2^N r0(M, ||H|| 2^-N) <= eps; N in [N0, N0 + 50], ties to smaller N.
 * Errors: EXPM_EINVAL, EXPM_ERANGE. */
int expm_choose_mn(double norm_h, double eps, int *M, int *N);

#ifdef __cplusplus
}
#endif
#endif /* EXPM_H */
