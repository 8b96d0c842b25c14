// Device helpers shared by the fused per-coordinate kernels and the
// persistent sweep kernel (gfx950, wave64).
#pragma once

#include "ss_internal.h"

namespace ss {
namespace dev {

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

// 1/x by the hardware's reciprocal estimate refined with Newton's iteration
// r <- r + r (1 - x r) (two steps in FP64, one in FP32): within a unit or two
// of the last place for the positive normal x of the transforms.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Sum over the wave, returned in every lane.
__device__ __forceinline__ double dpp_wave_sum(double x)
{
    return read_lane(dpp_incl_scan(x), kWave - 1);
}

// Inclusive wave-wide scan of NC doubles.
template <int NC>
__device__ __forceinline__ void wave_inclusive_scan(double (&x)[NC])
{
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = dpp_incl_scan(x[c]);
}

__device__ __forceinline__ double wave_sum(double x) { return dpp_wave_sum(x); }

// The same for floats (one DPP move per step).
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_float(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK,
                                                      0xF, BOUND_ZERO));
}
__device__ __forceinline__ float dpp_incl_scan(float x)
{
    x += dpp_float<0x111, 0xF, true>(x);
    x += dpp_float<0x112, 0xF, true>(x);
    x += dpp_float<0x114, 0xF, true>(x);
    x += dpp_float<0x118, 0xF, true>(x);
    x += dpp_float<0x142, 0xA, false>(x);
    x += dpp_float<0x143, 0xC, false>(x);
    return x;
}
__device__ __forceinline__ float dpp_wave_sum(float x)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dpp_incl_scan(x)),
                                                    kWave - 1));
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

// Sum of d log(s) over the events of one thread, kept as log(m) + k ln 2:
// s = f 2^e with f in [1/2, 1) contributes f^d to the product m and d e to
// the integer k, so a thread takes a single logarithm at the end.  f^d is
// formed by binary powering with the product renormalised after every
// multiplication (d = 1, almost every event, is one multiplication); m
// stays in [1/2, 1) between calls.  The exponents of add01 calls gather in
// a 32-bit counter that renorm_all folds into k (at most 32 calls of
// |e| <= 1100 in between).
struct LogSum {
    double m = 1.0;
    int64_t k = 0;
    int32_t k01 = 0;
    __device__ __forceinline__ void renorm(double &x, int64_t &kx)
    {
        kx += __builtin_amdgcn_frexp_exp(x);
        x = __builtin_amdgcn_frexp_mant(x);
    }
    __device__ __forceinline__ void add(double s, int d)
    {
        double f = __builtin_amdgcn_frexp_mant(s);
        k += (int64_t)__builtin_amdgcn_frexp_exp(s) * d;
        if (d == 1) {
            m *= f;
        } else {
            int64_t kf = 0;  // the base is f 2^kf
            for (uint32_t e = (uint32_t)d; e != 0u; e >>= 1) {
                if (e & 1u) {
                    m *= f;
                    k += kf;
                    renorm(m, k);
                }
                if (e > 1u) {
                    f *= f;
                    kf *= 2;
                    renorm(f, kf);
                }
            }
        }
        renorm(m, k);
    }
    // d in {0, 1}: no branch and no renormalisation (m stays above 2^-33
    // for up to 32 calls between renorm_all() calls)
    __device__ __forceinline__ void add01(double s, int d)
    {
        const double f = __builtin_amdgcn_frexp_mant(s);
        const int e = __builtin_amdgcn_frexp_exp(s);
        m *= d ? f : 1.0;
        k01 += d ? e : 0;
    }
    __device__ __forceinline__ void renorm_all()
    {
        k += k01;
        k01 = 0;
        renorm(m, k);
    }
    __device__ __forceinline__ double value() const
    {
        return (double)(k + k01) * 0.69314718055994530942 + log(m);
    }
};

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
constexpr uint8_t kFlagNext = 4;   // the next column has a non-zero here

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

// The column index arrays do not change while a kernel runs, so they are
// read through the constant address space: with uniform indices these are
// scalar loads, which count on their own counter, and vector loads issued
// around them (a tile's data) never wait for them or they for those.
template <typename T>
__device__ __forceinline__ T ld_const(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)(p);
}

__device__ __forceinline__ ColTile col_tile(const Column &col, int32_t j, int64_t chunk0,
                                            int64_t chunk1)
{
    ColTile ct;
    ct.cb = ld_const(col.col_ptr + j);
    const int32_t *cp = col.chunk_ptr + (int64_t)j * col.nchunk1;
    ct.lo = ld_const(cp + chunk0);
    ct.hi = ld_const(cp + chunk1);
    return ct;
}

// ---------------------------------------------------------------- pairs
// A published value travels as a 16-byte (value, tag) pair written and read
// with one agent-scope 16-byte access each, which the memory system performs
// as a unit, so a reader that sees the expected tag also sees the value and
// no separate flag or ordering wait is needed.  The tag carries the epoch of
// the step that wrote it.

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

// One 16-byte word, stored as st_pair stores a pair.
__device__ __forceinline__ void st_quad(u32x4 *p, u32x4 val)
{
    asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 4"
                 : : "v"(p), "v"(val) : "memory");
}

// Packed publications: N doubles in pub_words<N>() 16-byte words, three
// doubles in every two words, each word carrying the low 32 bits of the
// publication's tag in its last dword.  Every word is written and read with
// one 16-byte access, so a reader that sees the tag in all of them has a
// consistent snapshot; a publication takes about 2N/3 words instead of N
// (value, tag) pairs.  32-bit tags repeat only after 2^31 rounds or 2^30
// launches, long after a slot was last overwritten.
template <int N>
constexpr int pub_words()
{
    return (N / 3) * 2 + (N % 3 == 0 ? 0 : (N % 3 == 1 ? 1 : 2));
}

__device__ __forceinline__ uint32_t lo32(double v)
{
    return (uint32_t)(unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ uint32_t hi32(double v)
{
    return (uint32_t)((unsigned long long)__double_as_longlong(v) >> 32);
}
__device__ __forceinline__ double from32(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int N>
__device__ __forceinline__ void pub_pack(const double (&v)[N], uint32_t tag,
                                         u32x4 (&q)[pub_words<N>()])
{
    constexpr int G = N / 3, R = N % 3;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double d0 = v[3 * g], d1 = v[3 * g + 1], d2 = v[3 * g + 2];
        q[2 * g].x = lo32(d0);
        q[2 * g].y = hi32(d0);
        q[2 * g].z = lo32(d1);
        q[2 * g].w = tag;
        q[2 * g + 1].x = hi32(d1);
        q[2 * g + 1].y = lo32(d2);
        q[2 * g + 1].z = hi32(d2);
        q[2 * g + 1].w = tag;
    }
    if constexpr (R >= 1) {
        const double d0 = v[3 * G];
        const double d1 = R == 2 ? v[3 * G + (R == 2 ? 1 : 0)] : 0.0;
        q[2 * G].x = lo32(d0);
        q[2 * G].y = hi32(d0);
        q[2 * G].z = lo32(d1);
        q[2 * G].w = tag;
        if constexpr (R == 2) {
            q[2 * G + 1].x = hi32(d1);
            q[2 * G + 1].y = 0u;
            q[2 * G + 1].z = 0u;
            q[2 * G + 1].w = tag;
        }
    }
}

template <int N>
__device__ __forceinline__ void pub_unpack(const u32x4 (&q)[pub_words<N>()], double (&v)[N])
{
    constexpr int G = N / 3, R = N % 3;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        v[3 * g] = from32(q[2 * g].x, q[2 * g].y);
        v[3 * g + 1] = from32(q[2 * g].z, q[2 * g + 1].x);
        v[3 * g + 2] = from32(q[2 * g + 1].y, q[2 * g + 1].z);
    }
    if constexpr (R >= 1) v[3 * G] = from32(q[2 * G].x, q[2 * G].y);
    if constexpr (R == 2) v[3 * G + 1] = from32(q[2 * G].z, q[2 * G + 1].x);
}

template <int M>
__device__ __forceinline__ bool pub_tagged(const u32x4 (&q)[M], uint32_t tag)
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < M; ++c) ok = ok && q[c].w == tag;
    return ok;
}

// Loads NP consecutive pairs and waits for them (one statement, so the
// compiler cannot touch the destination registers before the wait).
template <int NP>
__device__ __forceinline__ void ld_pairs(const u32x4 *p, u32x4 (&r)[NP]);

template <>
__device__ __forceinline__ void ld_pairs<1>(const u32x4 *p, u32x4 (&r)[1])
{
    asm volatile("global_load_dwordx4 %0, %1, off sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<2>(const u32x4 *p, u32x4 (&r)[2])
{
    asm volatile("global_load_dwordx4 %0, %2, off sc1\n\t"
                 "global_load_dwordx4 %1, %2, off offset:16 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<3>(const u32x4 *p, u32x4 (&r)[3])
{
    asm volatile("global_load_dwordx4 %0, %3, off sc1\n\t"
                 "global_load_dwordx4 %1, %3, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %3, off offset:32 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<4>(const u32x4 *p, u32x4 (&r)[4])
{
    asm volatile("global_load_dwordx4 %0, %4, off sc1\n\t"
                 "global_load_dwordx4 %1, %4, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %4, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %4, off offset:48 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<6>(const u32x4 *p, u32x4 (&r)[6])
{
    asm volatile("global_load_dwordx4 %0, %6, off sc1\n\t"
                 "global_load_dwordx4 %1, %6, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %6, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %6, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %6, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %6, off offset:80 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<7>(const u32x4 *p, u32x4 (&r)[7])
{
    asm volatile("global_load_dwordx4 %0, %7, off sc1\n\t"
                 "global_load_dwordx4 %1, %7, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %7, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %7, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %7, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %7, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %7, off offset:96 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<8>(const u32x4 *p, u32x4 (&r)[8])
{
    asm volatile(
                 "global_load_dwordx4 %0, %8, off sc1\n\t"
                 "global_load_dwordx4 %1, %8, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %8, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %8, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %8, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %8, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %8, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %8, off offset:112 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<9>(const u32x4 *p, u32x4 (&r)[9])
{
    asm volatile("global_load_dwordx4 %0, %9, off sc1\n\t"
                 "global_load_dwordx4 %1, %9, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %9, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %9, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %9, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %9, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %9, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %9, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %9, off offset:128 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<15>(const u32x4 *p, u32x4 (&r)[15])
{
    asm volatile("global_load_dwordx4 %0, %15, off sc1\n\t"
                 "global_load_dwordx4 %1, %15, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %15, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %15, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %15, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %15, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %15, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %15, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %15, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %15, off offset:144 sc1\n\t"
                 "global_load_dwordx4 %10, %15, off offset:160 sc1\n\t"
                 "global_load_dwordx4 %11, %15, off offset:176 sc1\n\t"
                 "global_load_dwordx4 %12, %15, off offset:192 sc1\n\t"
                 "global_load_dwordx4 %13, %15, off offset:208 sc1\n\t"
                 "global_load_dwordx4 %14, %15, off offset:224 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11]), "=&v"(r[12]), "=&v"(r[13]), "=&v"(r[14])
                 : "v"(p)
                 : "memory");
}


template <>
__device__ __forceinline__ void ld_pairs<5>(const u32x4 *p, u32x4 (&r)[5])
{
    asm volatile(
                 "global_load_dwordx4 %0, %5, off sc1\n\t"
                 "global_load_dwordx4 %1, %5, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %5, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %5, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %5, off offset:64 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<10>(const u32x4 *p, u32x4 (&r)[10])
{
    asm volatile(
                 "global_load_dwordx4 %0, %10, off sc1\n\t"
                 "global_load_dwordx4 %1, %10, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %10, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %10, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %10, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %10, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %10, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %10, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %10, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %10, off offset:144 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs<11>(const u32x4 *p, u32x4 (&r)[11])
{
    asm volatile(
                 "global_load_dwordx4 %0, %11, off sc1\n\t"
                 "global_load_dwordx4 %1, %11, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %11, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %11, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %11, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %11, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %11, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %11, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %11, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %11, off offset:144 sc1\n\t"
                 "global_load_dwordx4 %10, %11, off offset:160 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10])
                 : "v"(p)
                 : "memory");
}

// Loads NP pairs at p and NP pairs 256 bytes further (two consecutive
// 16-pair slots) and waits for all of them.
template <int NP>
__device__ __forceinline__ void ld_pairs2(const u32x4 *p, u32x4 (&r0)[NP], u32x4 (&r1)[NP]);

template <>
__device__ __forceinline__ void ld_pairs2<9>(const u32x4 *p, u32x4 (&r0)[9],
                                               u32x4 (&r1)[9])
{
    asm volatile(
                 "global_load_dwordx4 %0, %18, off sc1\n\t"
                 "global_load_dwordx4 %1, %18, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %18, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %18, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %18, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %18, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %18, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %18, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %18, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %18, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %10, %18, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %11, %18, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %12, %18, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %13, %18, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %14, %18, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %15, %18, off offset:352 sc1\n\t"
                 "global_load_dwordx4 %16, %18, off offset:368 sc1\n\t"
                 "global_load_dwordx4 %17, %18, off offset:384 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r0[7]), "=&v"(r0[8]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6]), "=&v"(r1[7]), "=&v"(r1[8])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<15>(const u32x4 *p, u32x4 (&r0)[15],
                                               u32x4 (&r1)[15])
{
    asm volatile(
                 "global_load_dwordx4 %0, %30, off sc1\n\t"
                 "global_load_dwordx4 %1, %30, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %30, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %30, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %30, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %30, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %30, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %30, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %30, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %30, off offset:144 sc1\n\t"
                 "global_load_dwordx4 %10, %30, off offset:160 sc1\n\t"
                 "global_load_dwordx4 %11, %30, off offset:176 sc1\n\t"
                 "global_load_dwordx4 %12, %30, off offset:192 sc1\n\t"
                 "global_load_dwordx4 %13, %30, off offset:208 sc1\n\t"
                 "global_load_dwordx4 %14, %30, off offset:224 sc1\n\t"
                 "global_load_dwordx4 %15, %30, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %16, %30, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %17, %30, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %18, %30, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %19, %30, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %20, %30, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %21, %30, off offset:352 sc1\n\t"
                 "global_load_dwordx4 %22, %30, off offset:368 sc1\n\t"
                 "global_load_dwordx4 %23, %30, off offset:384 sc1\n\t"
                 "global_load_dwordx4 %24, %30, off offset:400 sc1\n\t"
                 "global_load_dwordx4 %25, %30, off offset:416 sc1\n\t"
                 "global_load_dwordx4 %26, %30, off offset:432 sc1\n\t"
                 "global_load_dwordx4 %27, %30, off offset:448 sc1\n\t"
                 "global_load_dwordx4 %28, %30, off offset:464 sc1\n\t"
                 "global_load_dwordx4 %29, %30, off offset:480 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r0[7]), "=&v"(r0[8]), "=&v"(r0[9]), "=&v"(r0[10]), "=&v"(r0[11]), "=&v"(r0[12]), "=&v"(r0[13]), "=&v"(r0[14]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6]), "=&v"(r1[7]), "=&v"(r1[8]), "=&v"(r1[9]), "=&v"(r1[10]), "=&v"(r1[11]), "=&v"(r1[12]), "=&v"(r1[13]), "=&v"(r1[14])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<4>(const u32x4 *p, u32x4 (&r0)[4],
                                               u32x4 (&r1)[4])
{
    asm volatile(
                 "global_load_dwordx4 %0, %8, off sc1\n\t"
                 "global_load_dwordx4 %1, %8, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %8, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %8, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %8, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %5, %8, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %6, %8, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %7, %8, off offset:304 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<5>(const u32x4 *p, u32x4 (&r0)[5],
                                               u32x4 (&r1)[5])
{
    asm volatile(
                 "global_load_dwordx4 %0, %10, off sc1\n\t"
                 "global_load_dwordx4 %1, %10, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %10, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %10, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %10, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %10, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %6, %10, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %7, %10, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %8, %10, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %9, %10, off offset:320 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<8>(const u32x4 *p, u32x4 (&r0)[8],
                                               u32x4 (&r1)[8])
{
    asm volatile(
                 "global_load_dwordx4 %0, %16, off sc1\n\t"
                 "global_load_dwordx4 %1, %16, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %16, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %16, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %16, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %16, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %16, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %16, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %16, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %9, %16, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %10, %16, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %11, %16, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %12, %16, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %13, %16, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %14, %16, off offset:352 sc1\n\t"
                 "global_load_dwordx4 %15, %16, off offset:368 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r0[7]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6]), "=&v"(r1[7])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<6>(const u32x4 *p, u32x4 (&r0)[6],
                                               u32x4 (&r1)[6])
{
    asm volatile(
                 "global_load_dwordx4 %0, %12, off sc1\n\t"
                 "global_load_dwordx4 %1, %12, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %12, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %12, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %12, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %12, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %12, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %7, %12, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %8, %12, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %9, %12, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %10, %12, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %11, %12, off offset:336 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<10>(const u32x4 *p, u32x4 (&r0)[10],
                                               u32x4 (&r1)[10])
{
    asm volatile(
                 "global_load_dwordx4 %0, %20, off sc1\n\t"
                 "global_load_dwordx4 %1, %20, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %20, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %20, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %20, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %20, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %20, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %20, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %20, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %20, off offset:144 sc1\n\t"
                 "global_load_dwordx4 %10, %20, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %11, %20, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %12, %20, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %13, %20, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %14, %20, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %15, %20, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %16, %20, off offset:352 sc1\n\t"
                 "global_load_dwordx4 %17, %20, off offset:368 sc1\n\t"
                 "global_load_dwordx4 %18, %20, off offset:384 sc1\n\t"
                 "global_load_dwordx4 %19, %20, off offset:400 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r0[7]), "=&v"(r0[8]), "=&v"(r0[9]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6]), "=&v"(r1[7]), "=&v"(r1[8]), "=&v"(r1[9])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<7>(const u32x4 *p, u32x4 (&r0)[7],
                                               u32x4 (&r1)[7])
{
    asm volatile(
                 "global_load_dwordx4 %0, %14, off sc1\n\t"
                 "global_load_dwordx4 %1, %14, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %14, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %14, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %14, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %14, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %14, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %14, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %8, %14, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %9, %14, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %10, %14, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %11, %14, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %12, %14, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %13, %14, off offset:352 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6])
                 : "v"(p)
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_pairs2<11>(const u32x4 *p, u32x4 (&r0)[11],
                                               u32x4 (&r1)[11])
{
    asm volatile(
                 "global_load_dwordx4 %0, %22, off sc1\n\t"
                 "global_load_dwordx4 %1, %22, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %22, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %22, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %22, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %22, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %22, off offset:96 sc1\n\t"
                 "global_load_dwordx4 %7, %22, off offset:112 sc1\n\t"
                 "global_load_dwordx4 %8, %22, off offset:128 sc1\n\t"
                 "global_load_dwordx4 %9, %22, off offset:144 sc1\n\t"
                 "global_load_dwordx4 %10, %22, off offset:160 sc1\n\t"
                 "global_load_dwordx4 %11, %22, off offset:256 sc1\n\t"
                 "global_load_dwordx4 %12, %22, off offset:272 sc1\n\t"
                 "global_load_dwordx4 %13, %22, off offset:288 sc1\n\t"
                 "global_load_dwordx4 %14, %22, off offset:304 sc1\n\t"
                 "global_load_dwordx4 %15, %22, off offset:320 sc1\n\t"
                 "global_load_dwordx4 %16, %22, off offset:336 sc1\n\t"
                 "global_load_dwordx4 %17, %22, off offset:352 sc1\n\t"
                 "global_load_dwordx4 %18, %22, off offset:368 sc1\n\t"
                 "global_load_dwordx4 %19, %22, off offset:384 sc1\n\t"
                 "global_load_dwordx4 %20, %22, off offset:400 sc1\n\t"
                 "global_load_dwordx4 %21, %22, off offset:416 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r0[0]), "=&v"(r0[1]), "=&v"(r0[2]), "=&v"(r0[3]), "=&v"(r0[4]), "=&v"(r0[5]), "=&v"(r0[6]), "=&v"(r0[7]), "=&v"(r0[8]), "=&v"(r0[9]), "=&v"(r0[10]), "=&v"(r1[0]), "=&v"(r1[1]), "=&v"(r1[2]), "=&v"(r1[3]), "=&v"(r1[4]), "=&v"(r1[5]), "=&v"(r1[6]), "=&v"(r1[7]), "=&v"(r1[8]), "=&v"(r1[9]), "=&v"(r1[10])
                 : "v"(p)
                 : "memory");
}



// Loads NC consecutive pairs at each of KQ addresses and waits for all of
// them (the look-back's predecessor windows).
template <int KQ, int NC>
__device__ __forceinline__ void ld_lb(const u32x4 *const (&p)[KQ], u32x4 (&r)[KQ][NC]);

template <>
__device__ __forceinline__ void ld_lb<4, 3>(const u32x4 *const (&p)[4],
                                               u32x4 (&r)[4][3])
{
    asm volatile(
                 "global_load_dwordx4 %0, %12, off sc1\n\t"
                 "global_load_dwordx4 %1, %12, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %12, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %13, off sc1\n\t"
                 "global_load_dwordx4 %4, %13, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %5, %13, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %6, %14, off sc1\n\t"
                 "global_load_dwordx4 %7, %14, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %8, %14, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %9, %15, off sc1\n\t"
                 "global_load_dwordx4 %10, %15, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %11, %15, off offset:32 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[1][0]), "=&v"(r[1][1]), "=&v"(r[1][2]), "=&v"(r[2][0]), "=&v"(r[2][1]), "=&v"(r[2][2]), "=&v"(r[3][0]), "=&v"(r[3][1]), "=&v"(r[3][2])
                 : "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<3, 3>(const u32x4 *const (&p)[3],
                                               u32x4 (&r)[3][3])
{
    asm volatile(
                 "global_load_dwordx4 %0, %9, off sc1\n\t"
                 "global_load_dwordx4 %1, %9, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %9, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %10, off sc1\n\t"
                 "global_load_dwordx4 %4, %10, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %5, %10, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %6, %11, off sc1\n\t"
                 "global_load_dwordx4 %7, %11, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %8, %11, off offset:32 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[1][0]), "=&v"(r[1][1]), "=&v"(r[1][2]), "=&v"(r[2][0]), "=&v"(r[2][1]), "=&v"(r[2][2])
                 : "v"(p[0]), "v"(p[1]), "v"(p[2])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<2, 2>(const u32x4 *const (&p)[2],
                                               u32x4 (&r)[2][2])
{
    asm volatile(
                 "global_load_dwordx4 %0, %4, off sc1\n\t"
                 "global_load_dwordx4 %1, %4, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %5, off sc1\n\t"
                 "global_load_dwordx4 %3, %5, off offset:16 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[1][0]), "=&v"(r[1][1])
                 : "v"(p[0]), "v"(p[1])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<2, 4>(const u32x4 *const (&p)[2],
                                               u32x4 (&r)[2][4])
{
    asm volatile(
                 "global_load_dwordx4 %0, %8, off sc1\n\t"
                 "global_load_dwordx4 %1, %8, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %8, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %8, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %9, off sc1\n\t"
                 "global_load_dwordx4 %5, %9, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %6, %9, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %7, %9, off offset:48 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[0][3]), "=&v"(r[1][0]), "=&v"(r[1][1]), "=&v"(r[1][2]), "=&v"(r[1][3])
                 : "v"(p[0]), "v"(p[1])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<2, 3>(const u32x4 *const (&p)[2],
                                               u32x4 (&r)[2][3])
{
    asm volatile(
                 "global_load_dwordx4 %0, %6, off sc1\n\t"
                 "global_load_dwordx4 %1, %6, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %6, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %7, off sc1\n\t"
                 "global_load_dwordx4 %4, %7, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %5, %7, off offset:32 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[1][0]), "=&v"(r[1][1]), "=&v"(r[1][2])
                 : "v"(p[0]), "v"(p[1])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<2, 6>(const u32x4 *const (&p)[2],
                                               u32x4 (&r)[2][6])
{
    asm volatile(
                 "global_load_dwordx4 %0, %12, off sc1\n\t"
                 "global_load_dwordx4 %1, %12, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %12, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %12, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %12, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %12, off offset:80 sc1\n\t"
                 "global_load_dwordx4 %6, %13, off sc1\n\t"
                 "global_load_dwordx4 %7, %13, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %8, %13, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %9, %13, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %10, %13, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %11, %13, off offset:80 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[0][3]), "=&v"(r[0][4]), "=&v"(r[0][5]), "=&v"(r[1][0]), "=&v"(r[1][1]), "=&v"(r[1][2]), "=&v"(r[1][3]), "=&v"(r[1][4]), "=&v"(r[1][5])
                 : "v"(p[0]), "v"(p[1])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<1, 2>(const u32x4 *const (&p)[1],
                                               u32x4 (&r)[1][2])
{
    asm volatile(
                 "global_load_dwordx4 %0, %2, off sc1\n\t"
                 "global_load_dwordx4 %1, %2, off offset:16 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1])
                 : "v"(p[0])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<1, 4>(const u32x4 *const (&p)[1],
                                               u32x4 (&r)[1][4])
{
    asm volatile(
                 "global_load_dwordx4 %0, %4, off sc1\n\t"
                 "global_load_dwordx4 %1, %4, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %4, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %4, off offset:48 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[0][3])
                 : "v"(p[0])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<1, 3>(const u32x4 *const (&p)[1],
                                               u32x4 (&r)[1][3])
{
    asm volatile(
                 "global_load_dwordx4 %0, %3, off sc1\n\t"
                 "global_load_dwordx4 %1, %3, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %3, off offset:32 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2])
                 : "v"(p[0])
                 : "memory");
}

template <>
__device__ __forceinline__ void ld_lb<1, 6>(const u32x4 *const (&p)[1],
                                               u32x4 (&r)[1][6])
{
    asm volatile(
                 "global_load_dwordx4 %0, %6, off sc1\n\t"
                 "global_load_dwordx4 %1, %6, off offset:16 sc1\n\t"
                 "global_load_dwordx4 %2, %6, off offset:32 sc1\n\t"
                 "global_load_dwordx4 %3, %6, off offset:48 sc1\n\t"
                 "global_load_dwordx4 %4, %6, off offset:64 sc1\n\t"
                 "global_load_dwordx4 %5, %6, off offset:80 sc1\n\t"
                 "s_waitcnt vmcnt(0)"
                 : "=&v"(r[0][0]), "=&v"(r[0][1]), "=&v"(r[0][2]), "=&v"(r[0][3]), "=&v"(r[0][4]), "=&v"(r[0][5])
                 : "v"(p[0])
                 : "memory");
}


// Polls NP pairs until all carry `tag`.  Returns false if the wait gave up
// or another workgroup already did.
template <int NP>
__device__ bool wait_pairs(const u32x4 *p, uint64_t tag, WsHeader *hdr, u32x4 (&r)[NP])
{
    uint32_t spins = 0;
    for (;;) {
        ld_pairs<NP>(p, r);
        bool ok = true;
#pragma unroll
        for (int c = 0; c < NP; ++c) ok = ok && pair_tag(r[c]) == tag;
        if (ok) return true;
        if ((++spins & 31u) == 0 && ld_relaxed_u32(&hdr->error)) return false;
        if (spins > kSpinLimit) {
            __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

}  // namespace dev
}  // namespace ss
