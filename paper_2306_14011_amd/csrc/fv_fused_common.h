// Device helpers shared by the fused stage kernels (2D and 3D): boundary
// index maps, wave reductions, buffer-descriptor access, DPP lane shifts and
// the XCD-aware block order.
#pragma once

#include "fv_internal.h"

namespace fvk {

constexpr int FW = 60;  // output columns per wave

// Index i of a cell within two of the axis (-2 <= i <= n + 1) mapped through
// the boundary kinds (0 periodic wrap, else transmissive clamp); anything
// beyond n + 1 maps to n - 1. Selects only, no division: for n >= 2 a wrap
// shifts by one period, and for n = 1 every index maps to 0.
__device__ __forceinline__ int map_index(int i, int n, int lo_kind, int hi_kind) {
    const int lo = lo_kind == 0 ? i + n : 0;
    const int hi = i > n + 1 ? n - 1 : (hi_kind == 0 ? i - n : n - 1);
    const int m = i < 0 ? lo : (i >= n ? hi : i);
    return n == 1 ? 0 : m;
}

// map_index with slip walls and inflow faces too (kinds 0 periodic, 1
// transmissive, 2 slip wall, 3 inflow): a wall reflects the index across the
// face (-1 -> 0, -2 -> 1; n -> n - 1, n + 1 -> n - 2); an inflow face's ghost
// positions read the nearest cell, whose value the caller then replaces by
// the given state. Anything beyond n + 1 maps to n - 1, as above.
__device__ __forceinline__ int map_index_bc(int i, int n, int lo_kind, int hi_kind) {
    const int lo = lo_kind == 0 ? i + n : (lo_kind == 2 ? -1 - i : 0);
    const int hi = i > n + 1 ? n - 1 : (hi_kind == 0 ? i - n : (hi_kind == 2 ? 2 * n - 1 - i : n - 1));
    const int m = i < 0 ? lo : (i >= n ? hi : i);
    return n == 1 ? 0 : m;
}

// Grid of the work item (uniform): largest g with work0 <= item.
__device__ __forceinline__ int find_grid(const FGrid* __restrict__ grids, int ngrids, int item) {
    int lo = 0, hi = ngrids - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grids[mid].work0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

// Buffer access with a wave-uniform descriptor (the grid's array), a per-lane
// 32-bit byte offset (the column) and a wave-uniform 32-bit byte offset (the
// variable and row): no per-lane 64-bit address arithmetic.
typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ __forceinline__ Rsrc grid_rsrc(const double* base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(unsigned int)bytes, 0x00020000);
}

__device__ __forceinline__ double ld_buf(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// Per-lane store offset for lanes with nothing to write: past the end of any
// buffer these kernels address (at most 2^31 bytes per descriptor used for
// stores, with scalar offsets below 2^31), so the buffer range check drops
// the store. Keeps lane-masked stores out of conditional blocks.
constexpr uint32_t DROP_OFFSET = 0x80000000u;

// NT: the store carries the non-temporal hint (cache policy bit 1). The 2D
// stage kernel's outputs are read a whole launch later, and keeping them out
// of L2's working set leaves room for the halo rows that neighbouring work
// items share (measured 1% faster); in 3D the hint measured slightly slower.
template <bool NT>
__device__ __forceinline__ void st_buf(Rsrc r, uint32_t voff, uint32_t soff, double x) {
    using T = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(T, x), r, (int)voff, (int)soff, NT ? 2 : 0);
}

// Value of lane l - 1 (UP) or l + 1 (down) of a double, by the whole-wave
// DPP shifts wave_shr:1 / wave_shl:1 on both halves (two VALU moves, no LDS
// round trip). The lane without a source (0 for UP, 63 otherwise) gets 0;
// only halo lanes see it, and their faces feed no output.
template <bool UP>
__device__ __forceinline__ double lane_shift1(double x) {
    const long long b = __double_as_longlong(x);
    int lo = (int)b, hi = (int)(b >> 32);
    constexpr int ctrl = UP ? 0x138 : 0x130;
    lo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The limited slope of a cell from its two differences for the limiter
// variant LIM of the fused kernels: 0 minmod, 3 van Leer (both symmetric).
template <int LIM>
__device__ __forceinline__ double limited_slope(double a, double b) {
    return LIM == 3 ? vanleer(a, b) : minmod(a, b);
}

// Block index with the hardware's round-robin spread over the 8 XCDs undone:
// block b runs on XCD b % 8, and the blocks of one XCD get a contiguous range
// of logical indices, so vertically adjacent segments (which share halo rows)
// are processed by the same XCD and its L2. A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace fvk
