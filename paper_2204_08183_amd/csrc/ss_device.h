// Device helpers shared by the fused per-coordinate kernels and the
// persistent sweep kernel (gfx950, wave64).
#pragma once

#include "ss_internal.h"

namespace ss {
namespace dev {

// Inclusive wave-wide scan of NC doubles (wave64 shuffles).
template <int NC>
__device__ __forceinline__ void wave_inclusive_scan(double (&x)[NC])
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double y = __shfl_up(x[c], off, kWave);
            if (lane >= off) x[c] += y;
        }
    }
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Block-wide sum of NC doubles in a fixed order; result valid in thread 0.
template <int NC, int BLOCK>
__device__ __forceinline__ void block_sum(double (&x)[NC], double *s_red)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = wave_sum(x[c]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) s_red[w * NC + c] = x[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int i = 0; i < NW; ++i) s += s_red[i * NC + c];
            x[c] = s;
        }
    }
}

// Loads IPT consecutive bytes of LDS (IPT in {4, 8, 16}) with one access.
template <int IPT>
__device__ __forceinline__ void lds_bytes(const uint8_t *p, uint8_t (&b)[IPT])
{
    if (IPT == 16) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) b[i] = (uint8_t)(w[i / 4] >> (8 * (i % 4)));
    } else if (IPT == 8) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        const uint32_t w[2] = {v.x, v.y};
#pragma unroll
        for (int i = 0; i < IPT; ++i) b[i] = (uint8_t)(w[i / 4] >> (8 * (i % 4)));
    } else {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
#pragma unroll
        for (int i = 0; i < IPT; ++i) b[i] = (uint8_t)(v >> (8 * i));
    }
}

// LDS flag bits per tile position.
constexpr uint8_t kFlagX = 1;      // column j has a non-zero here
constexpr uint8_t kFlagPatch = 2;  // the pending step changed e here

__device__ __forceinline__ void lds_flag_or(uint8_t *s_flag, int32_t r, uint8_t bit)
{
    atomicOr(reinterpret_cast<uint32_t *>(s_flag) + (r >> 2), (uint32_t)bit << (8 * (r & 3)));
}

// Per-tile view of one CSC column: offsets [lo, hi) into the column's rows.
struct ColTile {
    int64_t cb;  // column start in rows/vals
    int32_t lo;
    int32_t hi;
};

__device__ __forceinline__ ColTile col_tile(const Column &col, int32_t j, int64_t chunk0,
                                            int64_t chunk1)
{
    ColTile ct;
    ct.cb = col.col_ptr[j];
    const int32_t *cp = col.chunk_ptr + (int64_t)j * col.nchunk1;
    ct.lo = cp[chunk0];
    ct.hi = cp[chunk1];
    return ct;
}

}  // namespace dev
}  // namespace ss
