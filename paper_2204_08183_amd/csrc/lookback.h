// Decoupled look-back of the single-pass chained scans (Sec. 2.6), shared
// by the fused coordinate kernels and the adjoint scans.
#pragma once

#include "ss_device.h"
#include "ss_internal.h"

namespace ss {
namespace dev {

// ---------------------------------------------------------------- look-back
// Decoupled look-back (single-pass chained scan, Sec. 2.6).  A tile's slot
// holds its NC values packed into 16-byte words (three doubles per two
// words, ss_device.h), each word tagged with the low 32 bits of
// (epoch << 2) | state, state 1 = tile aggregate and 2 = inclusive prefix;
// the inclusive prefix overwrites the aggregate in place.  Each word is
// written and read as one 16-byte access, so a reader that sees all tags
// equal has a consistent snapshot (mixed tags: the slot is being
// overwritten, not ready yet), and one load brings a predecessor's state and
// value together: no flag word, no ordering wait on either side.  While the data stream
// saturates memory a round trip through the coherence point takes ~5 us, and
// one round trip instead of two (flags, then payloads) took the look-back
// from 11 to 5 us per tile at N = 2^27.
//
// Two levels.  Tiles form groups of kLbGroup = 64; the last tile of a full
// group also publishes the group's aggregate (as soon as its members'
// aggregates are visible) and later the group's inclusive prefix (its own).
// A tile's look-back runs over the sequence: its predecessors in its own
// group, then whole groups g-1, g-2, ...  With one level the inclusive
// prefixes advance by at most one window of tiles per round trip, which
// bounded the whole launch at large N; with groups one round reaches back
// up to 64 groups.
//
// Wave 0 looks back over 64 elements of that sequence per round: one load
// round trip for a round, the nearest inclusive prefix fixes which elements
// are needed, and only the needed ones that were not ready are polled
// again.  Every tile started earlier than its successors (workgroups start
// in index order on each XCD) and publishes its aggregate without waiting on
// anyone, and a group's aggregate waits only on its members, so every wait
// ends; it is bounded all the same.
constexpr int kLbSlot = 8;     // pairs per tile or group slot (128 bytes)

// The NC values packed into pub_words<NC>() words (ss_device.h) under the
// low 32 bits of tag; lane q of the calling wave stores word q.
template <int NC>
__device__ __forceinline__ void publish_pairs(u32x4 *slot, const double (&v)[NC],
                                              uint64_t tag)
{
    constexpr int NQ = pub_words<NC>();
    const int lane = lane_id();
    u32x4 q[NQ];
    pub_pack<NC>(v, (uint32_t)tag, q);
    // the words pass through an empty asm statement: a select chain over
    // the array itself is folded into an indexed load, which puts the array
    // in scratch memory
    u32x4 x = q[0];
#pragma unroll
    for (int c = 1; c < NQ; ++c) {
        u32x4 y = q[c];
        asm volatile("" : "+v"(y));
        x = lane == c ? y : x;
    }
    if (lane < NQ) st_quad(slot + lane, x);
}

// State of a snapshot of NQ words: all tags equal and of this launch (the
// low 30 bits of the epoch), else 0.
template <int NQ>
__device__ __forceinline__ uint32_t pairs_state(const u32x4 (&r)[NQ], uint64_t epoch)
{
    const uint32_t t0 = r[0].w;
    bool same = (t0 >> 2) == ((uint32_t)epoch & 0x3fffffffu);
#pragma unroll
    for (int c = 1; c < NQ; ++c) same = same && r[c].w == t0;
    return same ? (t0 & 3u) : 0u;
}

// Wave 0 only; the sum over the look-back sequence of `tile` is added to
// excl in every lane.  The sequence: tiles tile-1 .. tile-nin (nin tiles of
// the own group still to be summed), then groups g-1, g-2, ...; before group
// 0 the sequence ends in an empty inclusive prefix.  Returns false if the
// wait gave up (the error word is then set).
template <int NC>
__device__ bool look_back_seq(const u32x4 *lb, const u32x4 *glb, int32_t tile, int32_t nin,
                              int32_t g, uint64_t epoch, WsHeader *hdr, double (&excl)[NC],
                              uint64_t *lb_stats = nullptr)
{
    constexpr int NQ = pub_words<NC>();
    const int lane = lane_id();
    int32_t base = 0;  // sequence index of lane 0 in this round
    uint32_t spins = 0;
    uint32_t rounds = 0, waits = 0;
    for (;;) {
        ++rounds;
        // element base + lane: a tile of the own group, a group, or before
        // the start (then the lane reads its own tile's slot: one request per
        // wave, not a shared address every tile would hammer)
        const int32_t el = base + lane;
        const int32_t grp = g - 1 - (el - nin);
        const bool is_tile = el < nin;
        const bool before = !is_tile && grp < 0;
        const u32x4 *ptr = is_tile ? lb + (int64_t)(tile - 1 - el) * kLbSlot
                           : before ? lb + (int64_t)tile * kLbSlot
                                    : glb + (int64_t)grp * kLbSlot;
        double val[NC];
        uint32_t st;
        {
            u32x4 r[1][NQ];
            const u32x4 *pp[1] = {ptr};
            ld_lb<1, NQ>(pp, r);
            st = before ? (uint32_t)kStateInc : pairs_state<NQ>(r[0], epoch);
            pub_unpack<NC>(r[0], val);
#pragma unroll
            for (int c = 0; c < NC; ++c) val[c] = before ? 0.0 : val[c];
        }
        // nearest inclusive prefix: lowest lane holding one
        uint64_t m = __ballot(st == kStateInc);
        int fl = m ? __ffsll((unsigned long long)m) - 1 : kWave;
        // poll again only the needed elements that were not ready
        for (;;) {
            const bool pend = lane <= fl && st == 0u;
            if (!__any(pend)) break;
            if (pend) {
                u32x4 r[NQ];
                ld_pairs<NQ>(ptr, r);
                st = pairs_state<NQ>(r, epoch);
                pub_unpack<NC>(r, val);
            }
            ++waits;
            if (++spins > kSpinLimit) {
                if (lane == 0)
                    __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            // an element polled again may now hold its inclusive prefix: the
            // nearest one can only move closer
            m = __ballot(st == kStateInc);
            fl = m ? __ffsll((unsigned long long)m) - 1 : kWave;
            __builtin_amdgcn_s_sleep(2);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) excl[c] += wave_sum(lane <= fl ? val[c] : 0.0);
        if (fl < kWave) break;
        base += kWave;
    }
    if (lb_stats && lane == 0) *lb_stats = ((uint64_t)rounds << 32) | waits;
    return true;
}

// Wave 0 of a group's last tile: the sum of its group's other members
// (tiles tile-1 .. tile-nin, nin < 64) once all are visible, back to the
// nearest one holding its inclusive prefix if any; returns true in that
// case (sum is then the tile's whole exclusive prefix).  `ok` is cleared if
// the wait gave up (the error word is then set).
template <int NC>
__device__ bool group_members(const u32x4 *lb, int32_t tile, int32_t nin, uint64_t epoch,
                              WsHeader *hdr, double (&sum)[NC], bool &ok)
{
    constexpr int NQ = pub_words<NC>();
    const int lane = lane_id();
    const bool mine = lane < nin;
    const u32x4 *ptr = lb + (int64_t)(mine ? tile - 1 - lane : tile) * kLbSlot;
    double val[NC];
    uint32_t st;
    {
        u32x4 r[1][NQ];
        const u32x4 *pp[1] = {ptr};
        ld_lb<1, NQ>(pp, r);
        st = mine ? pairs_state<NQ>(r[0], epoch) : (uint32_t)kStateAgg;
        pub_unpack<NC>(r[0], val);
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] = mine ? val[c] : 0.0;
    }
    uint64_t m = __ballot(st == kStateInc);
    int fl = m ? __ffsll((unsigned long long)m) - 1 : kWave;
    uint32_t spins = 0;
    for (;;) {
        const bool pend = lane <= fl && st == 0u;
        if (!__any(pend)) break;
        if (pend) {
            u32x4 r[NQ];
            ld_pairs<NQ>(ptr, r);
            st = pairs_state<NQ>(r, epoch);
            pub_unpack<NC>(r, val);
        }
        if (++spins > kSpinLimit) {
            if (lane == 0)
                __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            return false;
        }
        m = __ballot(st == kStateInc);
        fl = m ? __ffsll((unsigned long long)m) - 1 : kWave;
        __builtin_amdgcn_s_sleep(2);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) sum[c] += wave_sum(lane <= fl ? val[c] : 0.0);
    return fl < kWave;
}

}  // namespace dev
}  // namespace ss
