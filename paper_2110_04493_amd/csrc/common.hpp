// Shared device/host declarations of the gfx950 expm library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace xpm {

constexpr int kWave = 64;

// Read-only device CSR view.
struct CsrView {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    const double *v;
};

// ---------------------------------------------------------------- wave ops
// All reductions use a fixed butterfly pattern, so results are bitwise
// reproducible from run to run.

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ double wave_min_f64(double x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ long long wave_sum_ll(long long x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

// Inclusive prefix sum across the 64 lanes.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        unsigned y = __shfl_up(x, d);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ long long wave_incl_scan_ll(long long x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        long long y = __shfl_up(x, d);
        if (l >= d) x += y;
    }
    return x;
}

// Maps a block index so that consecutive logical blocks run on the same XCD
// (the hardware hands block b to XCD b % 8).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks) {
    constexpr unsigned kXcd = 8;
    if (nblocks < kXcd) return b;
    unsigned per = nblocks / kXcd, rem = nblocks % kXcd, x = b % kXcd, j = b / kXcd;
    // XCDs x < rem own per+1 logical blocks, the others per.
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

// Work item of block b when the count is known only on the device: XCD
// b % 8 takes the contiguous range [x per, (x + 1) per), per = ceil(count /
// 8), in the order its blocks are dispatched, so that work items close in
// the list (which read the same operands) share that XCD's L2.  -1 for a
// surplus block; the grid needs at least 8 per blocks (count + 7).
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t count) {
    constexpr int64_t kXcd = 8;
    const int64_t per = (count + kXcd - 1) / kXcd, j = b / kXcd;
    if (j >= per) return -1;
    return (b % kXcd) * per + j;
}

}  // namespace xpm
