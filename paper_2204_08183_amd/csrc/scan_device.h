// Block-level pieces of the deterministic reduce-then-scan: a workgroup of
// SB threads scans a tile of ST = SB * SI items, each thread SI consecutive
// items, in a fixed order.  Device code only; each translation unit that
// includes it gets its own copy.
#pragma once

#include "ss_device.h"

namespace ss {
namespace {

using namespace dev;

template <typename T>
struct OpAdd {
    __device__ static T id() { return T(0); }
    __device__ static T op(T a, T b) { return a + b; }
};
template <typename T>
struct OpMul {
    __device__ static T id() { return T(1); }
    __device__ static T op(T a, T b) { return a * b; }
};

constexpr int SB = 256;          // scan block
constexpr int SI = 8;            // items per thread
constexpr int ST = SB * SI;      // items per scan tile

// Block-wide inclusive scan of SI items per thread (blocked arrangement)
// with a carry-in; returns the block total (carry excluded) to all threads.
template <typename T, typename Op>
__device__ T block_scan(T (&it)[SI], T carry, T *s_w)
{
    constexpr int NW = SB / kWave;
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    T run = Op::id();
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        run = Op::op(run, it[i]);
        it[i] = run;
    }
    T inc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc = Op::op(y, inc);
    }
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    T before = Op::id(), total = Op::id();
    for (int q = 0; q < NW; ++q) {
        if (q < w) before = Op::op(before, s_w[q]);
        total = Op::op(total, s_w[q]);
    }
    __syncthreads();
    // exclusive prefix of this thread = carry (+) wave prefix (+) lanes before
    T lanes_before = __shfl_up(inc, 1, kWave);
    T pre = Op::op(carry, before);
    if (lane > 0) pre = Op::op(pre, lanes_before);
#pragma unroll
    for (int i = 0; i < SI; ++i) it[i] = Op::op(pre, it[i]);
    return total;
}

template <typename T, bool REV>
__device__ __forceinline__ int64_t phys(int64_t i, int64_t m)
{
    return REV ? m - 1 - i : i;
}

// A thread's SI items are consecutive in memory (descending addresses when
// REV): a whole, 16-byte aligned run moves as 16-byte vectors, anything
// else item by item.
template <typename T, bool REV>
__device__ __forceinline__ const T *item_run(const T *p, int64_t base, int64_t m)
{
    if (base + SI > m) return nullptr;
    const T *r = p + (REV ? m - base - SI : base);
    return ((uintptr_t)r & 15u) == 0 ? r : nullptr;
}

template <typename T, typename Op, bool REV>
__device__ __forceinline__ void load_items(const T *in, int64_t base, int64_t m, T (&it)[SI])
{
    static_assert((SI * sizeof(T)) % 16 == 0, "a run of items is whole 16-byte vectors");
    constexpr int PV = 16 / sizeof(T);  // items per vector
    if (const T *r = item_run<T, REV>(in, base, m)) {
        const uint4 *v = reinterpret_cast<const uint4 *>(r);
#pragma unroll
        for (int q = 0; q < SI / PV; ++q) {
            union {
                uint4 u;
                T t[PV];
            } x;
            x.u = v[q];
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int i = q * PV + k;  // memory order
                it[REV ? SI - 1 - i : i] = x.t[k];
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int64_t l = base + i;
        it[i] = l < m ? in[phys<T, REV>(l, m)] : Op::id();
    }
}

template <typename T, bool REV>
__device__ __forceinline__ void store_items(T *out, int64_t base, int64_t m, const T (&it)[SI])
{
    constexpr int PV = 16 / sizeof(T);
    if (T *r = const_cast<T *>(item_run<T, REV>(out, base, m))) {
        uint4 *v = reinterpret_cast<uint4 *>(r);
#pragma unroll
        for (int q = 0; q < SI / PV; ++q) {
            union {
                uint4 u;
                T t[PV];
            } x;
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int i = q * PV + k;
                x.t[k] = it[REV ? SI - 1 - i : i];
            }
            v[q] = x.u;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int64_t l = base + i;
        if (l < m) out[phys<T, REV>(l, m)] = it[i];
    }
}

// Turns the inclusive values left by block_scan into exclusive ones: the
// exclusive value of an item is the inclusive value of the item before it,
// and the block's first item gets `carry`.
template <typename T>
__device__ void inclusive_to_exclusive(T (&it)[SI], T carry, T *s_last)
{
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const T prev = __shfl_up(it[SI - 1], 1, kWave);
    if (lane == kWave - 1) s_last[w] = it[SI - 1];
    __syncthreads();
    const T first = lane > 0 ? prev : (w > 0 ? s_last[w - 1] : carry);
    __syncthreads();
#pragma unroll
    for (int i = SI - 1; i > 0; --i) it[i] = it[i - 1];
    it[0] = first;
}

}  // namespace
}  // namespace ss
