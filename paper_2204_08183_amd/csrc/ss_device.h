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

// ---------------------------------------------------------------- DPP
// Wave64 scans and reductions of doubles on the VALU through DPP row shifts
// and row broadcasts (gfx9 family), one 32-bit half at a time; lanes a
// shift reads from outside the row, and rows the mask leaves out, add 0.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ double dpp_double(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xF,
                                               BOUND_ZERO);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF,
                                               BOUND_ZERO);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ double dpp_incl_scan(double x)
{
    x += dpp_double<0x111, 0xF, true>(x);  // row_shr:1
    x += dpp_double<0x112, 0xF, true>(x);  // row_shr:2
    x += dpp_double<0x114, 0xF, true>(x);  // row_shr:4
    x += dpp_double<0x118, 0xF, true>(x);  // row_shr:8
    x += dpp_double<0x142, 0xA, false>(x); // row_bcast:15 into rows 1 and 3
    x += dpp_double<0x143, 0xC, false>(x); // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ __forceinline__ double read_lane(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave, returned in every lane.
__device__ __forceinline__ double dpp_wave_sum(double x)
{
    return read_lane(dpp_incl_scan(x), kWave - 1);
}

// ---------------------------------------------------------------- pairs
// A published value travels as a 16-byte (value, tag) pair written and read
// with one agent-scope 16-byte access each, which the memory system performs
// as a unit, so a reader that sees the expected tag also sees the value and
// no separate flag or ordering wait is needed.  The tag carries the epoch of
// the step that wrote it.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 make_pair(double v, uint64_t tag)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    u32x4 r;
    r.x = (unsigned int)b;
    r.y = (unsigned int)(b >> 32);
    r.z = (unsigned int)tag;
    r.w = (unsigned int)(tag >> 32);
    return r;
}
__device__ __forceinline__ double pair_value(u32x4 r)
{
    return __longlong_as_double((long long)(((unsigned long long)r.y << 32) | r.x));
}
__device__ __forceinline__ uint64_t pair_tag(u32x4 r)
{
    return ((uint64_t)r.w << 32) | r.z;
}

// The s_nop after the store: a VMEM store of more than 64 bits must not have
// its data VGPRs overwritten by the next VALU instructions before it has
// read them (a GFX9-family hazard).  The compiler's hazard recognizer pads
// the stores it emits itself, but not one inside inline assembly, so the
// padding is part of the statement.
__device__ __forceinline__ void st_pair(u32x4 *p, double v, uint64_t tag)
{
    const u32x4 val = make_pair(v, tag);
    asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 4"
                 : : "v"(p), "v"(val) : "memory");
}

// Loads NP consecutive pairs (NP in {1, 3, 6}) and waits for them.
template <int NP>
__device__ __forceinline__ void ld_pairs(const u32x4 *p, u32x4 (&r)[NP])
{
    if (NP == 1) {
        asm volatile("global_load_dwordx4 %0, %1, off sc1\n\ts_waitcnt vmcnt(0)"
                     : "=&v"(r[0]) : "v"(p) : "memory");
    } else if (NP == 3) {
        asm volatile("global_load_dwordx4 %0, %3, off sc1\n\t"
                     "global_load_dwordx4 %1, %3, off offset:16 sc1\n\t"
                     "global_load_dwordx4 %2, %3, off offset:32 sc1\n\t"
                     "s_waitcnt vmcnt(0)"
                     : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]) : "v"(p) : "memory");
    } else {
        asm volatile("global_load_dwordx4 %0, %6, off sc1\n\t"
                     "global_load_dwordx4 %1, %6, off offset:16 sc1\n\t"
                     "global_load_dwordx4 %2, %6, off offset:32 sc1\n\t"
                     "global_load_dwordx4 %3, %6, off offset:48 sc1\n\t"
                     "global_load_dwordx4 %4, %6, off offset:64 sc1\n\t"
                     "global_load_dwordx4 %5, %6, off offset:80 sc1\n\t"
                     "s_waitcnt vmcnt(0)"
                     : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]),
                       "=&v"(r[5])
                     : "v"(p)
                     : "memory");
    }
}

}  // namespace dev
}  // namespace ss
