// Locality reordering: a symmetric permutation P applied as H' = P H P^T
// before the method runs, and E = P^T E' P after it.
//
// Every step of Algorithm 4.2 commutes with a symmetric permutation: the
// products, the Frobenius norms and the filter of Algorithm 4.1 (an entry is
// kept by its magnitude against a global threshold) give the permuted result
// up to the order of floating-point sums.  The permutation only changes which
// rows share a 16 x 16 tile.  In natural order a 2D grid puts 16 consecutive
// nodes on one grid line, so a tile row touches the whole band of every
// neighbouring line; grouping nodes into compact 2D cells roughly halves the
// tiles per block row and the matrix-core work of the late squarings.
//
// The order comes from graph distances alone, with no coordinates: breadth-
// first distances d1, d3 from two far-apart nodes (u1, the node farthest
// from node 0, and u3, the node farthest from both node 0 and u1) act as two
// coordinates.  Nodes are cut into strips of kStrip values of d1; each strip
// is walked along d3 (every other strip backwards) and, for one value of d3,
// by d1 and then index.  On a 2D mesh a run of 16 consecutive nodes is then
// a compact patch, and a patch's neighbours lie in few runs.  Graphs without
// such structure (small diameter, so very full cells) keep their order.
#include <string.h>

#include "plan.hpp"

namespace xpm {

constexpr int kBfsThreads = 1024;
constexpr int kCellMax = 256;      // largest cell the ordering accepts
constexpr int kLevelMax = 4096;    // largest level the level ordering accepts
constexpr int kStrip = 8;          // d1 values per strip
constexpr int kPermWaves = 4;        // output rows (waves) per workgroup
constexpr int kPermLdsWords = 1024;  // bit-map words per wave in LDS
constexpr int kPermCache = 32;       // mapped columns held per lane

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__device__ __forceinline__ long long wave_max_ll(long long x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    return x;
}

// Calls f(u) for every column u of G's row v.  The columns are loaded
// kNbrBatch at a time, all loads issued before the first use, so that a
// level of the search waits for one memory round trip per batch instead of
// one per edge.
constexpr int kNbrBatch = 8;

template <typename F>
__device__ __forceinline__ void for_neighbours(const CsrView &G, int v, F &&f) {
    const int64_t b = G.rp[v], e = G.rp[v + 1];
    for (int64_t p0 = b; p0 < e; p0 += kNbrBatch) {
        int u[kNbrBatch];
#pragma unroll
        for (int j = 0; j < kNbrBatch; ++j) u[j] = p0 + j < e ? G.ci[p0 + j] : -1;
#pragma unroll
        for (int j = 0; j < kNbrBatch; ++j)
            if (u[j] >= 0) f(u[j]);
    }
}

// G's rows in a fixed width of kEll slots per node (unused slots -1), so
// that a search level reads a node's neighbours in one round trip (two
// 16-byte loads) instead of two (the row bounds, then the columns); a row
// longer than kEll is marked with -2 in its first slot and read from G.
constexpr int kEll = 8;

__global__ void k_ell(CsrView G, int32_t *ell) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G.n) return;
    const int64_t b = G.rp[v], d = G.rp[v + 1] - b;
    int32_t r[kEll];
#pragma unroll
    for (int j = 0; j < kEll; ++j) r[j] = j < d ? G.ci[b + j] : -1;
    if (d > kEll) r[0] = -2;
    int4 *o = (int4 *)(ell + v * kEll);
    o[0] = make_int4(r[0], r[1], r[2], r[3]);
    o[1] = make_int4(r[4], r[5], r[6], r[7]);
}

template <typename F>
__device__ __forceinline__ void for_neighbours_ell(const CsrView &G, const int32_t *ell, int v,
                                                   F &&f) {
    const int4 *e = (const int4 *)(ell + (int64_t)v * kEll);
    const int4 x = e[0], y = e[1];
    if (x.x == -2) {
        for_neighbours(G, v, f);
        return;
    }
    const int u[kEll] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
#pragma unroll
    for (int j = 0; j < kEll; ++j)
        if (u[j] >= 0) f(u[j]);
}

// Breadth-first distances from *srcp over G's out-edges, in one workgroup
// (level-synchronous; the frontier of a mesh is small).  dist must hold -1.
// Nodes not reached get (largest distance + 1).  Writes res[0] = the node
// maximising dist (or min(dist, other) when other is given), smallest index
// on ties, and res[1] = the largest distance.
__global__ __launch_bounds__(kBfsThreads) void k_bfs(CsrView G, const int32_t *ell,
                                                     const int32_t *srcp, int32_t *dist,
                                                     int32_t *q0, int32_t *q1,
                                                     const int32_t *other, int32_t *res) {
    __shared__ int s_cnt[3];   // rotating frontier sizes, as in k_bfs_lds
    __shared__ long long s_best[kBfsThreads / kWave];
    __shared__ int s_unreached;
    const int tid = threadIdx.x;
    const int64_t n = G.n;
    if (tid == 0) {
        const int src = *srcp;
        atomicExch(&dist[src], 0);
        q0[0] = src;
        s_cnt[0] = 1;
        s_cnt[1] = 0;
        s_cnt[2] = 0;
        s_unreached = 0;
    }
    __syncthreads();
    int level = 0, c0 = 0, c1 = 1, c2 = 2;
    int32_t *cur = q0, *nxt = q1;
    for (;;) {
        const int size = s_cnt[c0];
        if (size == 0) break;
        for (int i = tid; i < size; i += kBfsThreads) {
            const int v = cur[i];
            for_neighbours_ell(G, ell, v, [&](int u) {
                // a stale -1 only costs a failed compare-and-swap
                if (dist[u] == -1 && atomicCAS(&dist[u], -1, level + 1) == -1)
                    nxt[atomicAdd(&s_cnt[c1], 1)] = u;
            });
        }
        if (tid == 0) s_cnt[c2] = 0;
        __syncthreads();
        const int t0 = c0;
        c0 = c1;
        c1 = c2;
        c2 = t0;
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
        ++level;
    }
    // level - 1 is the largest distance reached
    long long best = -1;
    for (int64_t v = tid; v < n; v += kBfsThreads) {
        int d = __hip_atomic_load(&dist[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (d < 0) {
            d = level;
            dist[v] = d;
            s_unreached = 1;
        }
        const int key = other ? min(d, other[v]) : d;
        const long long pk = ((long long)key << 32) | (long long)(0x7fffffff - (int)v);
        best = pk > best ? pk : best;
    }
    best = wave_max_ll(best);
    if (lane_id() == 0) s_best[tid / kWave] = best;
    __syncthreads();
    if (tid == 0) {
        long long b = s_best[0];
        for (int w = 1; w < kBfsThreads / kWave; ++w) b = s_best[w] > b ? s_best[w] : b;
        res[0] = 0x7fffffff - (int)(b & 0xffffffffll);
        res[1] = s_unreached ? level : level - 1;
    }
}

// The same breadth-first search with the visited set as a bit map in LDS
// (an LDS atomicOr marks a node instead of a compare-and-swap in memory) and
// the frontier queues in LDS; a frontier beyond kQCap nodes continues in
// the global queues at the same positions.  For n <= kBfsLdsNodes.
constexpr int kQCap = 4096;
constexpr int64_t kBfsLdsNodes = 200000;   // bit map + queues stay under 64 KB

__global__ __launch_bounds__(kBfsThreads) void k_bfs_lds(CsrView G, const int32_t *ell,
                                                         const int32_t *srcp, int32_t *dist,
                                                         int32_t *gq0, int32_t *gq1,
                                                         const int32_t *other, int32_t *res) {
    extern __shared__ uint32_t sm[];
    // frontier sizes rotate through three counters, so that one barrier per
    // level suffices: level L reads s_cnt[L % 3], counts the next frontier
    // into s_cnt[(L + 1) % 3] and clears s_cnt[(L + 2) % 3], last read (as
    // a size) before the previous level's barrier
    __shared__ int s_cnt[3], s_unreached;
    __shared__ long long s_best[kBfsThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t n = G.n;
    const int VW = (int)((n + 31) / 32);
    uint32_t *vis = sm;
    int32_t *lq0 = (int32_t *)(sm + VW), *lq1 = lq0 + kQCap;
    for (int i = tid; i < VW; i += kBfsThreads) vis[i] = 0u;
    __syncthreads();
    if (tid == 0) {
        const int src = *srcp;
        vis[src >> 5] |= 1u << (src & 31);
        dist[src] = 0;
        lq0[0] = src;
        s_cnt[0] = 1;
        s_cnt[1] = 0;
        s_cnt[2] = 0;
        s_unreached = 0;
    }
    __syncthreads();
    int level = 0, c0 = 0, c1 = 1, c2 = 2;
    int32_t *lcur = lq0, *lnxt = lq1, *gcur = gq0, *gnxt = gq1;
    for (;;) {
        const int size = s_cnt[c0];
        if (size == 0) break;
        for (int i = tid; i < size; i += kBfsThreads) {
            const int v = i < kQCap ? lcur[i] : gcur[i];
            for_neighbours_ell(G, ell, v, [&](int u) {
                const uint32_t bit = 1u << (u & 31);
                if (vis[u >> 5] & bit) return;
                if (atomicOr(&vis[u >> 5], bit) & bit) return;
                dist[u] = level + 1;
                const int pos = atomicAdd(&s_cnt[c1], 1);
                if (pos < kQCap) lnxt[pos] = u; else gnxt[pos] = u;
            });
        }
        if (tid == 0) s_cnt[c2] = 0;
        __syncthreads();
        const int t0 = c0;
        c0 = c1;
        c1 = c2;
        c2 = t0;
        int32_t *t = lcur;
        lcur = lnxt;
        lnxt = t;
        t = gcur;
        gcur = gnxt;
        gnxt = t;
        ++level;
    }
    long long best = -1;
    for (int64_t v = tid; v < n; v += kBfsThreads) {
        int d;
        if (vis[v >> 5] & (1u << (v & 31))) {
            d = __hip_atomic_load(&dist[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            d = level;
            dist[v] = d;
            s_unreached = 1;
        }
        const int key = other ? min(d, other[v]) : d;
        const long long pk = ((long long)key << 32) | (long long)(0x7fffffff - (int)v);
        best = pk > best ? pk : best;
    }
    best = wave_max_ll(best);
    if (lane_id() == 0) s_best[tid / kWave] = best;
    __syncthreads();
    if (tid == 0) {
        long long b = s_best[0];
        for (int w = 1; w < kBfsThreads / kWave; ++w) b = s_best[w] > b ? s_best[w] : b;
        res[0] = 0x7fffffff - (int)(b & 0xffffffffll);
        res[1] = s_unreached ? level : level - 1;
    }
}

// Cell of every node and the cell populations: strips of kStrip values of
// d1, each walked along d3, every other strip in the opposite direction;
// a cell is one value of d3 within a strip.
__global__ void k_cell_count(int64_t n, const int32_t *d1, const int32_t *d3, int64_t maxd3,
                             int64_t *cell, int64_t *cnt) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t strip = d1[v] / kStrip;
    const int64_t pos = (strip & 1) ? maxd3 - d3[v] : d3[v];
    const int64_t c = strip * (maxd3 + 1) + pos;
    cell[v] = c;
    atomicAdd((unsigned long long *)&cnt[c], 1ull);
}

__global__ void k_max_i64(const int64_t *a, int64_t n, int32_t *out) {
    __shared__ long long s[256 / kWave];
    long long m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = a[i] > m ? a[i] : m;
    m = wave_max_ll(m);
    if (lane_id() == 0) s[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long b = s[0];
        for (int w = 1; w < 256 / kWave; ++w) b = s[w] > b ? s[w] : b;
        atomicMax(out, (int)(b < 0x7fffffff ? b : 0x7fffffff));
    }
}

// The level ordering: cell = breadth-first level d1 (distance from u1).
__global__ void k_level_count(int64_t n, const int32_t *d1, int64_t *cell, int64_t *cnt) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t c = d1[v] < 0 ? 0 : d1[v];   // unreached nodes (other components) first
    cell[v] = c;
    atomicAdd((unsigned long long *)&cnt[c], 1ull);
}

__global__ void k_cell_scatter(int64_t n, const int64_t *cell, const int64_t *coff,
                               int64_t *cfill, int32_t *tmp) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t c = cell[v];
    const int64_t pos = coff[c] + (int64_t)atomicAdd((unsigned long long *)&cfill[c], 1ull);
    tmp[pos] = (int32_t)v;
}

// One wave per cell: members by ascending key (d1 for the strips, d3 for the
// levels), then node index (rank by counting).
__global__ void k_cell_sort(int64_t ncell, const int64_t *coff, const int32_t *tmp,
                            const int32_t *d1, int32_t *order, int32_t *newidx) {
    const int64_t c = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= ncell) return;
    const int64_t o = coff[c];
    const int k = (int)(coff[c + 1] - o);
    for (int j = lane_id(); j < k; j += kWave) {
        const int32_t x = tmp[o + j];
        const int32_t dx = d1[x];
        int r = 0;
        for (int i = 0; i < k; ++i) {
            const int32_t y = tmp[o + i], dy = d1[y];
            r += dy < dx || (dy == dx && y < x);
        }
        order[o + r] = x;
        newidx[x] = (int32_t)(o + r);
    }
}

// Permuted rows: output row r is input row src_row[r] with its columns
// mapped through colmap.  Per output row: its length and, when its column
// window is wider than the LDS bit map, the number of global words.
//
// ident: the rows of I + X instead (X square, colmap the inverse of src_row,
// so that input row s = src_row[r] keeps its diagonal at column s, mapped to
// r).  The diagonal takes 1 + x, is inserted as 1 where X has none, and is
// left out where 1 + x is exactly zero; the other entries stay as they are.
__global__ void k_perm_words(CsrView X, const int32_t *src_row, const int32_t *colmap,
                             int64_t *cnt, int64_t *gwords, int ident) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= X.n) return;
    const int32_t s = src_row[r];
    const int64_t b = X.rp[s], e = X.rp[s + 1];
    int mn = INT32_MAX, mx = -1;
    bool hasd = false, zerod = false;
    for (int64_t p = b + lane_id(); p < e; p += kWave) {
        const int32_t sc = X.ci[p];
        const int c = colmap[sc];
        mn = min(mn, c);
        mx = max(mx, c);
        if (ident && sc == s) {
            hasd = true;
            zerod = 1.0 + X.v[p] == 0.0;
        }
    }
    int64_t len = e - b;
    if (ident) {   // every lane is back from the loop
        if (__ballot(hasd) == 0) {
            mn = min(mn, (int)r);
            mx = max(mx, (int)r);
            ++len;
        } else if (__ballot(zerod) != 0) {
            --len;
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane_id() == 0) {
        cnt[r] = len;
        const int64_t W = mx < 0 ? 0 : (((int64_t)mx - (mn & ~31)) >> 5) + 1;
        gwords[r] = W > kPermLdsWords ? W : 0;
    }
}

// One wave per output row, kPermWaves rows per workgroup.  The mapped
// columns are marked in a bit map over the row's window; the rank of a
// column (prefix count + bits below it) is its position in the sorted output
// row.  Rows of up to kWave * kPermCache entries keep their mapped columns
// in registers between the passes.  emap (optional) receives, for every
// output entry, the index of its input entry (-1 for an inserted diagonal),
// tmap (optional), for every input entry, the index of its output entry (-1
// for a diagonal left out).  ident: the rows of I + X, as in k_perm_words.
__global__ __launch_bounds__(kWave * kPermWaves) void k_perm_rows(
    CsrView X, const int32_t *src_row, const int32_t *colmap, const int64_t *orp, int32_t *oci,
    double *ov, int64_t *emap, int64_t *tmap, const int64_t *gofs, uint2 *gbits, int cplx,
    int ident) {
    __shared__ uint2 lbits[kPermWaves][kPermLdsWords];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * kPermWaves + wv;
    if (r >= X.n) return;
    const int32_t s = src_row[r];
    const int64_t b = X.rp[s], e = X.rp[s + 1];
    if (e == b) {
        if (ident && lane == 0) {   // the row of I alone
            const int64_t q = orp[r];
            oci[q] = (int32_t)r;
            ov[q] = 1.0;
            if (emap) emap[q] = -1;
        }
        return;
    }
    const bool cached = e - b <= (int64_t)kWave * kPermCache;
    int cc[kPermCache];
    int mn = INT32_MAX, mx = -1;
    bool hasd = false, zerod = false;
    const int rd = (int)r;   // the diagonal's column in the output
    if (cached) {
#pragma unroll
        for (int j = 0; j < kPermCache; ++j) {
            const int64_t p = b + lane + (int64_t)kWave * j;
            cc[j] = p < e ? colmap[X.ci[p]] : -1;
            if (cc[j] >= 0) {
                mn = min(mn, cc[j]);
                mx = max(mx, cc[j]);
                if (ident && cc[j] == rd) {
                    hasd = true;
                    zerod = 1.0 + X.v[p] == 0.0;
                }
            }
        }
    } else {
        for (int64_t p = b + lane; p < e; p += kWave) {
            const int c = colmap[X.ci[p]];
            mn = min(mn, c);
            mx = max(mx, c);
            if (ident && c == rd) {
                hasd = true;
                zerod = 1.0 + X.v[p] == 0.0;
            }
        }
    }
    // ident: insert the diagonal (addd) or leave it out (a column no entry
    // takes otherwise: dskip); the window then spans r as k_perm_words's does
    bool addd = false;
    int dskip = -1;
    if (ident) {   // every lane is back from the loops
        addd = __ballot(hasd) == 0;
        if (addd) {
            mn = min(mn, rd);
            mx = max(mx, rd);
        } else if (__ballot(zerod) != 0) {
            dskip = rd;
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    const int lo = mn & ~31;
    const int64_t W = (((int64_t)mx - lo) >> 5) + 1;
    // The bit map lives in this wave's slice of LDS, or for very wide windows
    // in this row's slice of global scratch; every access goes through
    // device-coherent atomics so that the global case never reads a stale
    // cache line, and the wave's passes are separated by workgroup-scope
    // fences (which wait for its own stores).
    uint32_t *bits = W > kPermLdsWords ? (uint32_t *)(gbits + gofs[r]) : (uint32_t *)lbits[wv];
    auto ld = [](uint32_t *a) {
        return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto st = [](uint32_t *a, uint32_t v) {
        __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto pass_end = []() {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    };
    for (int64_t w = lane; w < W; w += kWave) {
        st(&bits[2 * w], 0u);
        st(&bits[2 * w + 1], 0u);
    }
    pass_end();
    auto mark = [&](int c) {
        if (c == dskip) return;
        const int d = c - lo;
        atomicOr(&bits[2 * (d >> 5)], 1u << (d & 31));
    };
    if (cached) {
#pragma unroll
        for (int j = 0; j < kPermCache; ++j)
            if (cc[j] >= 0) mark(cc[j]);
    } else {
        for (int64_t p = b + lane; p < e; p += kWave) mark(colmap[X.ci[p]]);
    }
    if (addd && lane == 0) mark(rd);
    pass_end();
    unsigned carry = 0;
    for (int64_t w0 = 0; w0 < W; w0 += kWave) {
        const int64_t w = w0 + lane;
        const unsigned pc = w < W ? __popc(ld(&bits[2 * w])) : 0u;
        const unsigned inc = wave_incl_scan(pc);
        if (w < W) st(&bits[2 * w + 1], carry + inc - pc);
        carry += __shfl(inc, kWave - 1);
    }
    pass_end();
    const int64_t ob = orp[r];
    auto slot = [&](int c) {
        const int d = c - lo;
        const uint32_t wx = ld(&bits[2 * (d >> 5)]), wy = ld(&bits[2 * (d >> 5) + 1]);
        return ob + wy + __popc(wx & ((1u << (d & 31)) - 1u));
    };
    auto place = [&](int c, int64_t p) {
        if (c == dskip) {
            if (tmap) tmap[p] = -1;
            return;
        }
        const int64_t q = slot(c);
        oci[q] = c;
        if (cplx)   // complex values: pairs of doubles
            ((double2 *)ov)[q] = ((const double2 *)X.v)[p];
        else
            ov[q] = ident && c == rd ? 1.0 + X.v[p] : X.v[p];
        if (emap) emap[q] = p;
        if (tmap) tmap[p] = q;
    };
    if (addd && lane == 0) {
        const int64_t q = slot(rd);
        oci[q] = rd;
        ov[q] = 1.0;
        if (emap) emap[q] = -1;
    }
    if (cached) {
#pragma unroll
        for (int j = 0; j < kPermCache; ++j)
            if (cc[j] >= 0) place(cc[j], b + lane + (int64_t)kWave * j);
    } else {
        for (int64_t p = b + lane; p < e; p += kWave) place(colmap[X.ci[p]], p);
    }
}

__global__ void k_scatter_map(const double *src, const int64_t *map, int64_t m, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) dst[map[i]] = src[i];
}

__global__ void k_gather_map(const double *src, const int64_t *map, int64_t m, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        const int64_t j = map[i];
        dst[i] = j >= 0 ? src[j] : 0.0;
    }
}

static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

namespace host {

// The level ordering of G (a Cuthill-McKee-like order): nodes by their
// breadth-first level from the far node u1, within a level by the distance
// from u3 and then index.  An edge joins nodes of one level or of adjacent
// levels, so the bandwidth l of the reordered matrix is at most four times
// the largest level.  With `force` unset it is taken only when that bound
// is below the bandwidth of the given order.
static int level_order(expm_plan_s &P, CsrView G, int64_t nnz, int64_t maxd1, bool force,
                       bool *active) {
    hipStream_t st = P.st;
    const int64_t n = G.n, ncell = maxd1 + 1;
    int32_t *rb = (int32_t *)P.ro_rb.p, *d1 = (int32_t *)P.ro_d1.p, *d3 = (int32_t *)P.ro_d3.p,
            *q0 = (int32_t *)P.ro_q0.p;
    CHK(ensure(P, P.ro_cell, sizeof(int64_t) * n));
    CHK(ensure(P, P.ro_cnt, sizeof(int64_t) * (ncell + 1)));
    CHK(ensure(P, P.ro_off, sizeof(int64_t) * (ncell + 1)));
    CHK(ensure(P, P.bands, sizeof(long long) * 2));
    int64_t *cell = (int64_t *)P.ro_cell.p, *cnt = (int64_t *)P.ro_cnt.p,
            *off = (int64_t *)P.ro_off.p;
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (ncell + 1), st));
    HIPCHK(hipMemsetAsync(rb + 10, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_level_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, d1, cell, cnt);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_max_i64, dim3(blocks_for(ncell, 256) < 1024 ? blocks_for(ncell, 256)
                                                                       : 1024),
                       dim3(256), 0, st, cnt, ncell, rb + 10);
    HIPCHK(hipGetLastError());
    HIPCHK(band_of(G, nullptr, (long long *)P.bands.p, st));
    CHK(scan(P, cnt, off, ncell));
    int32_t *hb = (int32_t *)P.host;
    HIPCHK(hipMemcpyAsync(hb + 10, rb + 10, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hb + 12, P.bands.p, sizeof(long long) * 2, hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    const int64_t maxlevel = hb[10];
    long long lb[2];
    memcpy(lb, hb + 12, sizeof lb);
    const long long band = lb[0] == LLONG_MIN ? 0 : lb[0] + lb[1];
    (void)nnz;
    if (maxlevel > kLevelMax) return EXPM_OK;               // sorting a level would not pay
    if (!force && 4 * maxlevel >= band) return EXPM_OK;    // the given order is as narrow
    CHK(ensure(P, P.order, sizeof(int32_t) * n));
    CHK(ensure(P, P.newidx, sizeof(int32_t) * n));
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (ncell + 1), st));
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, cell, off,
                       cnt, q0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_cell_sort, dim3(blocks_for(ncell, 4)), dim3(256), 0, st, ncell, off,
                       q0, d3, (int32_t *)P.order.p, (int32_t *)P.newidx.p);
    HIPCHK(hipGetLastError());
    *active = true;
    P.ordering = 2;
    return EXPM_OK;
}

// Computes the cell ordering of G's pattern into P.order (new -> old) and
// P.newidx (old -> new); *active = false when no ordering applies (then
// nothing is permuted).  mode 1: the strips, else the level ordering when
// it narrows the band; mode 2: the level ordering.
int compute_reorder(expm_plan_s &P, CsrView G, int64_t nnz, int mode, bool *active) {
    hipStream_t st = P.st;
    const int64_t n = G.n;
    *active = false;
    if (n < 2) return EXPM_OK;
    CHK(ensure(P, P.ro_rb, sizeof(int32_t) * 16));
    CHK(ensure(P, P.ro_d0, sizeof(int32_t) * n));
    CHK(ensure(P, P.ro_d1, sizeof(int32_t) * n));
    CHK(ensure(P, P.ro_d3, sizeof(int32_t) * n));
    CHK(ensure(P, P.ro_q0, sizeof(int32_t) * n));
    CHK(ensure(P, P.ro_q1, sizeof(int32_t) * n));
    int32_t *rb = (int32_t *)P.ro_rb.p, *d0 = (int32_t *)P.ro_d0.p, *d1 = (int32_t *)P.ro_d1.p,
            *d3 = (int32_t *)P.ro_d3.p, *q0 = (int32_t *)P.ro_q0.p, *q1 = (int32_t *)P.ro_q1.p;
    HIPCHK(hipMemsetAsync(rb, 0, sizeof(int32_t) * 16, st));
    CHK(ensure(P, P.ro_ell, sizeof(int32_t) * kEll * n));
    int32_t *ell = (int32_t *)P.ro_ell.p;
    hipLaunchKernelGGL(k_ell, dim3(blocks_for(n, 256)), dim3(256), 0, st, G, ell);
    HIPCHK(hipGetLastError());
    auto bfs = [&](const int32_t *srcp, int32_t *dist, const int32_t *other, int32_t *res) {
        if (n <= kBfsLdsNodes) {
            const size_t lds = sizeof(uint32_t) * ((n + 31) / 32) + sizeof(int32_t) * 2 * kQCap;
            hipLaunchKernelGGL(k_bfs_lds, dim3(1), dim3(kBfsThreads), lds, st, G, ell, srcp, dist,
                               q0, q1, other, res);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, dist, n, -1);
        hipLaunchKernelGGL(k_bfs, dim3(1), dim3(kBfsThreads), 0, st, G, ell, srcp, dist, q0, q1,
                           other, res);
        return hipGetLastError();
    };
    // rb: [0] node 0 | [1..2] u1, max d0 | [3..4] u3 = argmax min(d0, d1), max d1 |
    //     [7..8] -, max d3
    HIPCHK(bfs(rb + 0, d0, nullptr, rb + 1));
    HIPCHK(bfs(rb + 1, d1, d0, rb + 3));
    HIPCHK(bfs(rb + 3, d3, nullptr, rb + 7));
    int32_t *hb = (int32_t *)P.host;
    HIPCHK(hipMemcpyAsync(hb, rb, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    const int64_t maxd1 = hb[4], maxd3 = hb[8];
    if (mode == 2) return level_order(P, G, nnz, maxd1, true, active);
    const int64_t ncell = (maxd1 / kStrip + 1) * (maxd3 + 1);
    // path-like: the level ordering, if it narrows the band
    if (ncell > 4 * n + 1024) return level_order(P, G, nnz, maxd1, false, active);
    CHK(ensure(P, P.ro_cell, sizeof(int64_t) * n));
    CHK(ensure(P, P.ro_cnt, sizeof(int64_t) * (ncell + 1)));
    CHK(ensure(P, P.ro_off, sizeof(int64_t) * (ncell + 1)));
    int64_t *cell = (int64_t *)P.ro_cell.p, *cnt = (int64_t *)P.ro_cnt.p,
            *off = (int64_t *)P.ro_off.p;
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (ncell + 1), st));
    hipLaunchKernelGGL(k_cell_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, d1, d3, maxd3,
                       cell, cnt);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_max_i64, dim3(blocks_for(ncell, 256) < 1024 ? blocks_for(ncell, 256)
                                                                       : 1024),
                       dim3(256), 0, st, cnt, ncell, rb + 9);
    HIPCHK(hipGetLastError());
    CHK(scan(P, cnt, off, ncell));
    HIPCHK(hipMemcpyAsync(hb + 9, rb + 9, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    // no 2D structure: the level ordering, if it narrows the band
    if (hb[9] > kCellMax) return level_order(P, G, nnz, maxd1, false, active);
    CHK(ensure(P, P.order, sizeof(int32_t) * n));
    CHK(ensure(P, P.newidx, sizeof(int32_t) * n));
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (ncell + 1), st));
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, cell, off,
                       cnt, q0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_cell_sort, dim3(blocks_for(ncell, 4)), dim3(256), 0, st, ncell, off,
                       q0, d1, (int32_t *)P.order.p, (int32_t *)P.newidx.p);
    HIPCHK(hipGetLastError());
    *active = true;
    P.ordering = 1;
    return EXPM_OK;
}

// The row pointers of the permuted X (of I + X with ident) into orp (n + 1
// entries), the global bit-map words of the widest rows, and both totals
// read back (one wait): *total output entries, *gwords words.
int permute_count(expm_plan_s &P, CsrView X, const int32_t *src_row, const int32_t *colmap,
                  int64_t *orp, bool ident, int64_t *total, int64_t *gwords) {
    hipStream_t st = P.st;
    const int64_t n = X.n;
    CHK(ensure(P, P.ro_pcnt, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.ro_pw, sizeof(int64_t) * (n + 1)));
    CHK(ensure(P, P.ro_pofs, sizeof(int64_t) * (n + 1)));
    int64_t *pc = (int64_t *)P.ro_pcnt.p, *pw = (int64_t *)P.ro_pw.p,
            *pofs = (int64_t *)P.ro_pofs.p;
    hipLaunchKernelGGL(k_perm_words, dim3(blocks_for(n, 4)), dim3(256), 0, st, X, src_row, colmap,
                       pc, pw, ident ? 1 : 0);
    HIPCHK(hipGetLastError());
    CHK(scan(P, pc, orp, n));
    CHK(scan(P, pw, pofs, n));
    int64_t *hl = (int64_t *)P.host;
    HIPCHK(hipMemcpyAsync(hl, orp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hl + 1, pofs + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHK(sync(P));
    *total = hl[0];
    *gwords = hl[1];
    return EXPM_OK;
}

// The entries of the permuted X (of I + X with ident) into oci, ov on the
// row pointers orp that permute_count gave (gwords from the same call).
int permute_write(expm_plan_s &P, CsrView X, int64_t nnz, const int32_t *src_row,
                  const int32_t *colmap, const int64_t *orp, int32_t *oci, double *ov,
                  int64_t *emap, int64_t *tmap, int64_t gwords, bool cplx, bool ident) {
    if (ident && cplx) return fail(EXPM_ENOTIMPL, "permute_write: I + X is real only");
    const int64_t n = X.n;
    CHK(ensure(P, P.ro_gbits, sizeof(uint2) * (gwords + 1)));
    if (nnz > 0 || (ident && n > 0)) {
        hipLaunchKernelGGL(k_perm_rows, dim3((unsigned)((n + kPermWaves - 1) / kPermWaves)),
                           dim3(kWave * kPermWaves), 0, P.st, X, src_row, colmap, orp, oci, ov,
                           emap, tmap, (const int64_t *)P.ro_pofs.p, (uint2 *)P.ro_gbits.p,
                           cplx ? 1 : 0, ident ? 1 : 0);
        HIPCHK(hipGetLastError());
    }
    return EXPM_OK;
}

// Output CSR (orp, oci, ov; caller-allocated, nnz entries) whose row r is
// row src_row[r] of X with columns mapped by colmap, sorted.
int permute_csr(expm_plan_s &P, CsrView X, int64_t nnz, const int32_t *src_row,
                const int32_t *colmap, int64_t *orp, int32_t *oci, double *ov, int64_t *emap,
                bool cplx) {
    int64_t total = 0, gw = 0;
    CHK(permute_count(P, X, src_row, colmap, orp, false, &total, &gw));
    return permute_write(P, X, nnz, src_row, colmap, orp, oci, ov, emap, nullptr, gw, cplx,
                         false);
}

int gather_map(expm_plan_s &P, const double *src, const int64_t *map, int64_t m, double *dst) {
    if (m <= 0) return EXPM_OK;
    hipLaunchKernelGGL(k_gather_map, dim3(blocks_for(m, 256)), dim3(256), 0, P.st, src, map, m,
                       dst);
    HIPCHK(hipGetLastError());
    return EXPM_OK;
}

int scatter_map(expm_plan_s &P, const double *src, const int64_t *map, int64_t m, double *dst) {
    if (m <= 0) return EXPM_OK;
    hipLaunchKernelGGL(k_scatter_map, dim3(blocks_for(m, 256)), dim3(256), 0, P.st, src, map, m,
                       dst);
    HIPCHK(hipGetLastError());
    return EXPM_OK;
}

}  // namespace host
}  // namespace xpm
