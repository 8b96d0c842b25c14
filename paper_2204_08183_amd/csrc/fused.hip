// Fused coordinate kernels for gfx950: the sparse update of X beta (step
// (1) of Sec. 2.7), the single-pass tuple scan with decoupled look-back,
// the element-wise transform with the event counts and the reduction
// (steps (2)-(4), fused as in Fig. 2), and the coordinate update in the
// last tile (Fig. 3's conditional kernel, Secs. 2.3-2.4).
//
// Data layout (sorted order = decreasing observed time):
//   e[n]  f64      exp(X beta), dense
//   d8[n] u8       events per tie run at the run's last position (255 =
//                  read d32[n] instead)
//   Fine-Gray also w_comp[n] f64 (competing-event weight 1/G(y)) and
//   g_end[n] f64 (G(y) at each position).
//   Column j: rows/vals of the CSC design in sorted positions plus a chunk
//   index, so each tile finds its non-zeros with two loads.
//
// A tile is BLOCK*IPT consecutive positions, one workgroup per tile.  The
// tuple is (e, e x, e x^2) for Cox and additionally (e w, e x w, e x^2 w)
// for Fine-Gray; its prefix at the end of every tie run gives S0, S1, S2
// (Sec. 2.7).  The Fine-Gray suffix over later competing events is the
// grand total minus the inclusive prefix of the weighted components; the
// totals come from a short reduction pass launched just before.
#include <algorithm>
#include <type_traits>

#include "lookback.h"
#include "ss_device.h"

namespace ss {

namespace {

using namespace dev;

// Phase timestamps per tile for performance analysis builds only
// (-DSS_TRACE_TIMES): 100 MHz real-time counter, 8 slots per tile, written
// behind the regular workspace.
#ifdef SS_TRACE_TIMES
#define SS_TRACE(ws, tile, slot)                                                   \
    do {                                                                           \
        if (threadIdx.x == 0)                                                      \
            trace_base(ws)[(tile) * 8 + (slot)] = __builtin_amdgcn_s_memrealtime(); \
    } while (0)
#else
#define SS_TRACE(ws, tile, slot) do { } while (0)
#endif

// Polls a publication of NV packed values (publish_pairs) until all its
// words carry `tag`, then unpacks them; false if the wait gave up (then the
// error word is set) or another wait already did.
template <int NV>
__device__ __forceinline__ bool poll_pairs(const u32x4 *p, uint64_t tag, WsHeader *hdr,
                                           double (&v)[NV])
{
    constexpr int NQ = pub_words<NV>();
    uint32_t spins = 0;
    for (;;) {
        u32x4 r[NQ];
        ld_pairs<NQ>(p, r);
        if (pub_tagged<NQ>(r, (uint32_t)tag)) {
            pub_unpack<NV>(r, v);
            return true;
        }
        if (++spins > kSpinLimit || ((spins & 31u) == 0 && ld_relaxed_u32(&hdr->error))) {
            __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// ------------------------------------------------------ partial sums
// Two-level reduction of the per-tile partial sums, in a fixed order (so
// the result does not depend on timing): every tile publishes its NR sums
// as packed words (slots of SLOT words); the last tile of each group of kGroup
// tiles waits for its group (wave 0, one tile per lane) and publishes the
// group's sums; the last tile of the launch waits for the groups and adds
// them.  Only tiles with smaller indices are ever waited for.
//
// tile_sum: the calling tile's sums (valid in every thread).  In the last
// tile, `total` (thread 0) receives the launch total; a wait that gives up
// sets the error word and leaves its share out.  s_red: NR + BLOCK/64 * NR
// doubles of LDS.
template <int BLOCK, int NR, int SLOT>
__device__ void reduce_partials(u32x4 *part, u32x4 *gpart, int64_t tile, int64_t ntiles,
                                uint64_t tag, WsHeader *hdr, const double (&tile_sum)[NR],
                                double (&total)[NR], double *s_red)
{
    static_assert(NR <= SLOT, "a slot holds the sums");
    const int lane = lane_id();
    const int tid = threadIdx.x;
    const bool last = tile == ntiles - 1;
    const bool leader = last || (tile % kGroup) == kGroup - 1;
    if (tid < kWave) {
        if (!leader) {
            publish_pairs<NR>(part + tile * SLOT, tile_sum, tag);
        } else {
            // wave 0 of a group leader: tiles g0 .. tile, this tile's own
            // sums from registers
            const int64_t g0 = tile - tile % kGroup;
            const int64_t t = g0 + lane;
            double v[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) v[c] = 0.0;
            if (t < tile) {
                double r[NR];
                if (poll_pairs<NR>(part + t * SLOT, tag, hdr, r)) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) v[c] = r[c];
                }
            } else if (t == tile) {
#pragma unroll
                for (int c = 0; c < NR; ++c) v[c] = tile_sum[c];
            }
            double g[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) g[c] = dpp_wave_sum(v[c]);
            if (!last) publish_pairs<NR>(gpart + (tile / kGroup) * SLOT, g, tag);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < NR; ++c) s_red[c] = g[c];
            }
        }
    }
    if (!last) return;
    __syncthreads();
    // the last tile: groups 0 .. ngroups-2 from memory, its own from LDS
    const int64_t ngroups = tile / kGroup + 1;
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    for (int64_t q = tid; q < ngroups - 1; q += BLOCK) {
        double r[NR];
        if (!poll_pairs<NR>(gpart + q * SLOT, tag, hdr, r)) break;
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] += r[c];
    }
    double own[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) own[c] = s_red[c];
    block_sum<NR, BLOCK>(acc, s_red + NR);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c) total[c] = acc[c] + own[c];
    }
}

// Last tile: g', g'', the likelihood or the coordinate update from the
// launch totals (thread 0), then the launch epoch moves on.
//
// CARRY (Fine-Gray, 0/1 design): tot[3], tot[4] are sum e w x_next and
// sum e w x_j x_next over the launch, fgw = (sum e w, sum e w x_j) its
// totals; the coordinate's step s multiplies e by exp(s) where x_j = 1, so
// the totals of column jnext over the updated e are sum e w + expm1(s)
// sum e w x_j (m = 0) and tot[3] + expm1(s) tot[4] (m = 1, 2), stored for the
// next launch.
template <int BLOCK, int NR, bool CARRY>
__device__ void finish(const FusedCall &a, const WsView &ws, uint64_t epoch,
                       const double (&tot)[NR], const double *fgw, double *s_red)
{
    // beta' c and the penalty's sum (|beta_q| for l1, beta_q^2 for l2)
    double all[2] = {0.0, 0.0};
    if (a.beta_ll) {
        for (int64_t q = threadIdx.x; q < a.p; q += BLOCK) {
            const double b = a.beta_ll[q];
            all[0] += b * a.c[q];
            all[1] += a.obj_penalty == SS_PENALTY_L2 ? b * b : fabs(b);
        }
    }
    block_sum<2, BLOCK>(all, s_red);
    if (threadIdx.x == 0) {
        const double A = tot[0], B = tot[1], L = tot[2];
        if (a.beta_ll) {
            const double l = all[0] - L;
            if (a.obj_penalty >= 0) {
                double pi = 0.0;
                if (a.obj_penalty == SS_PENALTY_L1) pi = -a.obj_lambda * all[1];
                if (a.obj_penalty == SS_PENALTY_L2) pi = -all[1] / (2.0 * a.obj_lambda);
                a.out[0] = l + pi;
                a.out[1] = l;
                a.out[2] = pi;
            } else {
                a.out[0] = l;
            }
        } else {
            const double g1 = a.c[a.j] - A;
            const double g2 = -B;
            a.out[0] = g1;
            a.out[1] = g2;
            a.out[2] = L;
            if (a.ccd) {
                ccd_apply(g1, g2, a.penalty, a.lambda, a.beta + a.j,
                          a.delta + a.j, a.steps + a.j);
            }
            if constexpr (CARRY) {
                const double em = expm1(a.steps[a.j]);
                const double t1 = tot[3] + em * tot[4];
                ws.hdr->fg_tot[0] = fgw[0] + em * fgw[1];
                ws.hdr->fg_tot[1] = t1;
                ws.hdr->fg_tot[2] = t1;
            }
        }
        if (a.err_out) a.err_out[0] = ld_relaxed_u32(&ws.hdr->error) ? 1.0 : 0.0;
        // every tile has read the epoch (it published a partial tagged with it)
        st_relaxed_u64(&ws.hdr->epoch, epoch + 1);
    }
}

// Position map of a tile (BLOCK threads, IPT elements each): the tile is
// R = IPT / CONSEC rows of BLOCK * CONSEC positions, and in every row a
// thread holds CONSEC consecutive positions.  Element i = q * CONSEC + k of
// thread tid sits at position
//   q * BLOCK * CONSEC + tid * CONSEC + k.
// Streaming alone, 8 doubles per thread per row (a wave's 16-byte loads then
// cover whole 128-byte lines) reads at 6.5 TB/s against 4.6 TB/s for 16;
// in this kernel, though, the second row costs registers (3 workgroups per
// CU instead of 4) and the tile waits on its look-back far longer than on
// its loads, so one row of 16 measured faster (0.89 ms against 0.93 ms at
// N = 2^27).  kConsecMax keeps the choice in one place.
#ifndef SS_FG_G_LDS
#define SS_FG_G_LDS 1
#endif
#ifndef SS_TF_GROUP
#define SS_TF_GROUP 4
#endif
constexpr int kTfGroup = SS_TF_GROUP;  // run ends evaluated together (branch-free path)
#ifndef SS_CONSEC_MAX
#define SS_CONSEC_MAX 16
#endif
constexpr int kConsecMax = SS_CONSEC_MAX;
template <int IPT>
struct TileMap {
    static constexpr int CONSEC = IPT < kConsecMax ? IPT : kConsecMax;
    static constexpr int R = IPT / CONSEC;
};

template <int BLOCK, int IPT>
__device__ __forceinline__ int32_t tile_pos(int i, int t)
{
    constexpr int C = TileMap<IPT>::CONSEC;
    return (i / C) * (BLOCK * C) + t * C + (i % C);
}

// Lane-major LDS slot of tile position r: [i * BLOCK + owner thread].
template <int BLOCK, int IPT>
__device__ __forceinline__ int32_t lds_slot(int32_t r)
{
    constexpr int C = TileMap<IPT>::CONSEC;
    const int32_t q = r / (BLOCK * C), rem = r % (BLOCK * C);
    return (q * C + rem % C) * BLOCK + rem / C;
}

// Clears a tile's LDS flags and (VALS) its values of column j, so that a
// position absent from the column reads x = 0.
template <int BLOCK, int TILE, bool VALS>
__device__ __forceinline__ void clear_tile_lds(uint8_t *s_flag, double *s_xv)
{
    const int tid = threadIdx.x;
    uint32_t *f32 = reinterpret_cast<uint32_t *>(s_flag);
    for (int i = tid; i < TILE / 4; i += BLOCK) f32[i] = 0u;
    if constexpr (VALS) {
        double2 *x2 = reinterpret_cast<double2 *>(s_xv);
        for (int i = tid; i < TILE / 2; i += BLOCK) x2[i] = make_double2(0.0, 0.0);
    }
}

// Stages one tile (positions [t0, t0+cnt)): e (patched by the pending step
// of column jprev, which is also written back to eta and e), the weights w
// (Fine-Gray) and the event counts d (one byte each, element i in byte i%4
// of word i/4) go to registers.  Column j: a 0/1 column leaves a bit per
// element in a register (returned: bit i for element i); a valued column
// leaves its values in LDS at s_xv[i * BLOCK + tid] (lane-major, free of
// bank conflicts; 0 where the column has no entry, and the returned bits
// carry nothing).  All independent loads are issued together; the sparse
// 0/1 column and the patch travel through LDS flag bytes (position order).
// s_flag and s_xv must be zero and visible on entry; ends after one
// workgroup barrier.
// NEXT: the 0/1 column jnext also goes to the flags; its bits are returned
// in *nbits.
template <int BLOCK, int IPT, bool WANT_W, bool VALS, bool PREV, bool WANT_D,
          bool NEXT = false, typename ET = double>
__device__ __forceinline__ uint32_t stage_tile(const FusedCall &a, int64_t t0, int64_t cnt,
                                               int64_t chunk0, int64_t chunk1,
                                               uint8_t *s_flag, double *s_xv, double *s_ep,
                                               ET (&ev)[IPT],
                                               double (&wv)[WANT_W ? IPT : 1],
                                               uint32_t (&dw)[(IPT + 3) / 4],
                                               uint32_t *nbits = nullptr)
{
    static_assert(IPT <= 32 && (IPT & (IPT - 1)) == 0 && IPT >= 4,
                  "IPT: a power of two from 4 to 32");
    constexpr bool E32 = std::is_same<ET, float>::value;
    static_assert(!E32 || (!PREV && !NEXT), "FP32 e: gradient and Hessian only");
    constexpr int TILE = BLOCK * IPT;
    constexpr int C = TileMap<IPT>::CONSEC;
    constexpr int R = TileMap<IPT>::R;
    const int tid = threadIdx.x;
    ColTile cj = {0, 0, 0};
    if (a.j >= 0) cj = col_tile(a.col, a.j, chunk0, chunk1);
    ColTile cnext = {0, 0, 0};
    if (NEXT) cnext = col_tile(a.col, a.jnext, chunk0, chunk1);
    ColTile cprev = {0, 0, 0};
    double step_prev = 0.0;
    if (PREV) {
        step_prev = *a.step_prev;
        cprev = col_tile(a.col, a.jprev, chunk0, chunk1);
    }
    const bool full = cnt == TILE;
    if (full) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t rb = t0 + (int64_t)q * BLOCK * C + (int64_t)tid * C;
            if constexpr (E32) {
                const float4 *ep = reinterpret_cast<const float4 *>(a.e32 + rb);
#pragma unroll
                for (int h = 0; h < C / 4; ++h) {
                    const float4 v = ep[h];
                    ev[q * C + 4 * h] = v.x;
                    ev[q * C + 4 * h + 1] = v.y;
                    ev[q * C + 4 * h + 2] = v.z;
                    ev[q * C + 4 * h + 3] = v.w;
                }
            } else {
                const double2 *ep = reinterpret_cast<const double2 *>(a.e + rb);
#pragma unroll
                for (int h = 0; h < C / 2; ++h) {
                    const double2 v = ep[h];
                    ev[q * C + 2 * h] = v.x;
                    ev[q * C + 2 * h + 1] = v.y;
                }
            }
            if (WANT_D) {
                if (C >= 8) {
                    const uint2 *dp = reinterpret_cast<const uint2 *>(a.d8 + rb);
#pragma unroll
                    for (int h = 0; h < C / 8; ++h) {
                        const uint2 dd = dp[h];
                        dw[q * (C / 4) + 2 * h] = dd.x;
                        dw[q * (C / 4) + 2 * h + 1] = dd.y;
                    }
                } else {
                    dw[q] = *reinterpret_cast<const uint32_t *>(a.d8 + rb);
                }
            }
            if (WANT_W) {
                const double2 *wp = reinterpret_cast<const double2 *>(a.w_comp + rb);
#pragma unroll
                for (int h = 0; h < C / 2; ++h) {
                    const double2 v = wp[h];
                    wv[q * C + 2 * h] = v.x;
                    wv[q * C + 2 * h + 1] = v.y;
                }
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < (IPT + 3) / 4; ++q) dw[q] = 0u;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int64_t k = t0 + tile_pos<BLOCK, IPT>(i, tid);
            const bool ok = k < a.n;
            if constexpr (E32) ev[i] = ok ? a.e32[k] : 0.f;
            else ev[i] = ok ? a.e[k] : 0.0;
            if (WANT_D && ok) dw[i / 4] |= (uint32_t)a.d8[k] << (8 * (i % 4));
            if (WANT_W) wv[i] = ok ? a.w_comp[k] : 0.0;
        }
    }
    // a column with a non-zero at every position of a full tile is read
    // straight from its value array (no scatter, no flags)
    const bool dense = full && (int64_t)(cj.hi - cj.lo) == cnt &&
                       (!VALS || ((uintptr_t)(a.col.vals + cj.cb + cj.lo) & 15u) == 0);
    if (dense) {
        if (VALS) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double2 *vp = reinterpret_cast<const double2 *>(
                    a.col.vals + cj.cb + cj.lo + q * BLOCK * C + tid * C);
#pragma unroll
                for (int h = 0; h < C / 2; ++h) {
                    const double2 v = vp[h];
                    s_xv[(q * C + 2 * h) * BLOCK + tid] = v.x;
                    s_xv[(q * C + 2 * h + 1) * BLOCK + tid] = v.y;
                }
            }
        }
    } else {
        for (int32_t o = cj.lo + tid; o < cj.hi; o += BLOCK) {
            const int32_t r = (int32_t)(a.col.rows[cj.cb + o] - t0);
            if (VALS) s_xv[lds_slot<BLOCK, IPT>(r)] = a.col.vals[cj.cb + o];
            else lds_flag_or(s_flag, r, kFlagX);
        }
    }
    if (NEXT) {
        for (int32_t o = cnext.lo + tid; o < cnext.hi; o += BLOCK)
            lds_flag_or(s_flag, (int32_t)(a.col.rows[cnext.cb + o] - t0), kFlagNext);
    }
    if (PREV && step_prev != 0.0) {
        for (int32_t o = cprev.lo + tid; o < cprev.hi; o += BLOCK) {
            const int32_t k = a.col.rows[cprev.cb + o];
            const double x = VALS ? a.col.vals[cprev.cb + o] : 1.0;
            const double et = a.eta[k] + x * step_prev;
            const double en = exp(et);
            a.eta[k] = et;
            a.e[k] = en;
            s_ep[k - t0] = en;
            lds_flag_or(s_flag, (int32_t)(k - t0), kFlagPatch);
        }
    }
    __syncthreads();
    uint32_t xbits = 0u;
    uint32_t pbits = 0u;
    uint32_t qbits = 0u;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        uint8_t fl[C];
        lds_bytes<C>(s_flag + q * BLOCK * C + tid * C, fl);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            xbits |= (uint32_t)(fl[k] & kFlagX) << (q * C + k);
            pbits |= (uint32_t)((fl[k] & kFlagPatch) ? 1u : 0u) << (q * C + k);
            if (NEXT) qbits |= (uint32_t)((fl[k] & kFlagNext) ? 1u : 0u) << (q * C + k);
        }
    }
    if (NEXT) *nbits = qbits;
    if (dense) xbits = IPT == 32 ? ~0u : (1u << IPT) - 1u;
    if (PREV) {
#pragma unroll
        for (int i = 0; i < IPT; ++i)
            if ((pbits >> i) & 1u) ev[i] = s_ep[tile_pos<BLOCK, IPT>(i, tid)];
    }
    return xbits;
}

// x of column j at element i of this thread (see stage_tile).
template <int BLOCK, bool VALS>
__device__ __forceinline__ double x_at(uint32_t xbits, int i, const double *s_xv)
{
    if (VALS) return s_xv[i * BLOCK + threadIdx.x];  // 0 where absent
    return ((xbits >> i) & 1u) ? 1.0 : 0.0;
}

// The tuple of Sec. 2.7 at one position, added to running sums S.  Cox:
// (e, e x, e x^2); Fine-Gray adds (e w, e x w, e x^2 w).  With a 0/1 column
// e x^2 = e x, so only the distinct components are carried (NX of them):
// Cox 2 or 3, Fine-Gray 4 or 6; EX, EXX, EW, EXW, EXXW index them (EXX and
// EXXW fall back on EX and EXW for 0/1 columns).
template <int BLOCK, int MODEL, bool VALS>
struct Tuple {
    static constexpr bool FG = MODEL == SS_FINE_GRAY;
    static constexpr int NX = (VALS ? 3 : 2) * (FG ? 2 : 1);
    static constexpr int EX = 1;
    static constexpr int EXX = VALS ? 2 : 1;
    static constexpr int EW = VALS ? 3 : 2;
    static constexpr int EXW = VALS ? 4 : 3;
    static constexpr int EXXW = VALS ? 5 : 3;
    template <typename AT>
    __device__ static __forceinline__ void add(AT (&S)[NX], AT e, uint32_t xbits, int i,
                                               const double *s_xv, double w)
    {
        if constexpr (VALS) {
            // positions absent from the column hold x = 0 in LDS
            const AT x = (AT)s_xv[i * BLOCK + threadIdx.x];
            const AT ex = e * x;
            S[0] += e;
            S[1] += ex;
            S[2] += ex * x;
            if constexpr (FG) {
                const AT ew = e * (AT)w;
                const AT exw = ew * x;
                S[3] += ew;
                S[4] += exw;
                S[5] += exw * x;
            }
        } else {
            const bool nz = (xbits >> i) & 1u;
            S[0] += e;
            S[1] += nz ? e : (AT)0;
            if constexpr (FG) {
                const AT ew = e * (AT)w;
                S[2] += ew;
                S[3] += nz ? ew : (AT)0;
            }
        }
    }
};

// The fused scan -> transform -> reduce kernel (one coordinate).
// MODEL: SS_COX (3 tuple components) or SS_FINE_GRAY (6).  PREV: apply the
// pending step of column jprev to eta and e first (step (1) of Sec. 2.7).
// CARRY (Fine-Gray, 0/1 design): the weighted totals of column j were
// carried by the previous launch, and this launch carries those of column
// jnext (two more partial sums, see finish).
//
// ET: storage type of e (float: FP32 storage, read from a.e32).  F32S (with
// float storage): the sums inside a tile (thread-serial and wave scans), the
// transform and the per-thread sums of the reduction in FP32; what crosses a
// tile boundary (aggregates, the look-back prefix, the tile partial sums)
// in FP64, and each run end's prefix is the FP64 carry plus the FP32
// in-tile prefix.  Without F32S every sum is FP64.
template <int BLOCK, int IPT, int MODEL, bool VALS, bool PREV, bool CARRY = false,
          typename ET = double, bool F32S = false>
__global__ __launch_bounds__(BLOCK) void k_fused(FusedCall a, WsView ws, int64_t ntiles)
{
    constexpr int TILE = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    constexpr int NR = CARRY ? 5 : 3;  // partial sums per tile
    static_assert(TILE % SS_CHUNK == 0, "tile must be whole chunks");
    static_assert(!CARRY || (MODEL == SS_FINE_GRAY && !VALS), "carry: Fine-Gray, 0/1 design");
    static_assert(!F32S || std::is_same<ET, float>::value, "FP32 sums need FP32 storage");
    // arithmetic type of the sums inside a tile
    using AT = typename std::conditional<F32S, float, double>::type;
    using Tx = Tuple<BLOCK, MODEL, VALS>;
    constexpr int NX = Tx::NX;  // distinct tuple components

    __shared__ __attribute__((aligned(16))) uint8_t s_flag[TILE];
    __shared__ __attribute__((aligned(16))) double s_xv[VALS ? TILE : 1];
    // G(Y) of the tile (Fine-Gray) and the patched e of the pending update
    // (PREV) share one array: the patch is consumed during staging, and with
    // PREV the copy of G is only started after that
    constexpr bool kGLds = SS_FG_G_LDS && MODEL == SS_FINE_GRAY;
    __shared__ __attribute__((aligned(16))) double s_eg[(PREV || kGLds) ? TILE : 1];
    double *const s_ep = s_eg;
    double *const s_g = s_eg;
    __shared__ double s_wsum[TileMap<IPT>::R][NW][NX];
    __shared__ double s_excl[NX];
    __shared__ double s_red[NW * NR + NR];
    __shared__ double s_tsum[NR];
    __shared__ double s_fgw[2];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;

    // ---- 1. the tile is the workgroup index: workgroups start in index
    // order on each XCD, so every predecessor a tile waits for has started
    // (the waits are bounded all the same); clear the LDS flags and values
    // meanwhile.  Each wave reads the launch's epoch itself, so no barrier
    // waits on that load and the tile's data loads go out at once; the epoch
    // changes only at the end of the launch's last tile, after every tile has
    // used it.
    SS_TRACE(ws, (int64_t)blockIdx.x, 0);
    const uint64_t epoch = ld_relaxed_u64(&ws.hdr->epoch);
    if (tid == 0 && a.clear_error && blockIdx.x == 0) st_relaxed_u32(&ws.hdr->error, 0u);
    clear_tile_lds<BLOCK, TILE, VALS>(s_flag, s_xv);
    __syncthreads();
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * TILE;
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = t0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + TILE / SS_CHUNK, nchunk);
    const int64_t cnt = min((int64_t)TILE, a.n - t0);

    // ---- 2-4. tile data, column j and the pending update into registers
    constexpr int C = TileMap<IPT>::CONSEC;
    constexpr int R = TileMap<IPT>::R;
    // Fine-Gray: G(Y) of a full tile goes straight from memory into LDS
    // (no registers), issued with the staging loads, so the transform finds
    // it there at the run ends instead of waiting on loads of its own after
    // the look-back.  Lane l of wave v puts its elements 2u, 2u + 1 at
    // s_g[v * IPT * 64 + u * 128 + 2 l].  A partial last tile reads G at its
    // run ends.
    const bool g_lds = kGLds && cnt == TILE;
    if (!PREV && g_lds) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int h = 0; h < C / 2; ++h) {
                const int u = q * (C / 2) + h;
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void *>(a.g_end + t0 + (int64_t)q * BLOCK * C +
                                              (int64_t)tid * C + 2 * h),
                    (__attribute__((address_space(3))) void *)(s_g + w * (IPT * kWave) +
                                                               u * (2 * kWave)),
                    16, 0, 0);
            }
        }
    }
    ET ev[IPT];
    double wv[MODEL == SS_FINE_GRAY ? IPT : 1];
    uint32_t dw[(IPT + 3) / 4];  // event counts, one byte per element
    uint32_t nbits = 0u;         // CARRY: column jnext, one bit per element
    const uint32_t xbits =
        stage_tile<BLOCK, IPT, MODEL == SS_FINE_GRAY, VALS, PREV, true, CARRY, ET>(
            a, t0, cnt, chunk0, chunk1, s_flag, s_xv, s_ep, ev, wv, dw, &nbits);
    if constexpr (PREV && kGLds) {
        // every thread has read its patches: the array takes G now, loaded
        // by waves 1.. for all waves (wave 0's loads would hold up its
        // look-back, which waits on its own memory counter)
        __syncthreads();
        if (g_lds && w != 0) {
            for (int m = w - 1; m < NW * (IPT / 2); m += NW - 1) {
                const int v = m / (IPT / 2), u = m % (IPT / 2);
                const int q = u / (C / 2), h = u % (C / 2);
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void *>(a.g_end + t0 + (int64_t)q * BLOCK * C +
                                              (int64_t)(v * kWave + lane) * C + 2 * h),
                    (__attribute__((address_space(3))) void *)(s_g + v * (IPT * kWave) +
                                                               u * (2 * kWave)),
                    16, 0, 0);
            }
        }
    }
    SS_TRACE(ws, tile, 1);

    // ---- 5. thread totals per row and their wave scans (which are also the
    // scan inside the tile: the thread's exclusive prefix within the tile is
    // kept across the look-back, NX values per row), the tile's aggregate
    AT texcl[R][NX];
    double agg[NX];
    {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            AT run[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) run[c] = (AT)0;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int i = q * C + k;
                Tx::add(run, (AT)ev[i], xbits, i, s_xv, wv[MODEL == SS_FINE_GRAY ? i : 0]);
            }
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                const AT inc = dpp_incl_scan(run[c]);
                texcl[q][c] = inc - run[c];
                if (lane == kWave - 1) s_wsum[q][w][c] = (double)inc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            double t = 0.0;
            AT done = (AT)0;  // rows before q
#pragma unroll
            for (int q = 0; q < R; ++q) {
                AT before = (AT)0, row = (AT)0;
#pragma unroll
                for (int v = 0; v < NW; ++v) {
                    const double sv = s_wsum[q][v][c];
                    if (v < w) before += (AT)sv;
                    row += (AT)sv;
                    t += sv;
                }
                texcl[q][c] += done + before;
                done += row;
            }
            agg[c] = t;
        }
    }

    // ---- 6. decoupled look-back for the tile's exclusive prefix
    SS_TRACE(ws, tile, 2);
    if (w == 0) {
        u32x4 *slot = ws.lb + tile * kLbSlot;
        double ex[NX];
        uint64_t *lbs = nullptr;
#ifdef SS_TRACE_TIMES
        if (tile != ntiles - 1)
            lbs = trace_base(ws) + tile * 8 + 5;
#endif
#pragma unroll
        for (int c = 0; c < NX; ++c) ex[c] = 0.0;
        const int32_t ti = (int32_t)tile;
        const int32_t g = ti / kLbGroup, pos = ti % kLbGroup;
        // the last tile of a full group publishes the group's slot (the last
        // tile of the launch has no reader)
        const bool leader = pos == kLbGroup - 1 && tile != ntiles - 1;
        if (tile == 0) {
            publish_pairs<NX>(slot, agg, (epoch << 2) | kStateInc);
        } else {
            publish_pairs<NX>(slot, agg, (epoch << 2) | kStateAgg);
            SS_TRACE(ws, tile, 6);
            // a wait that gives up has set the error word; the launch still
            // runs to its end
            if (!leader) {
                (void)look_back_seq<NX>(ws.lb, ws.glb, ti, pos, g, epoch, ws.hdr, ex, lbs);
            } else {
                bool ok = true;
                if (!group_members<NX>(ws.lb, ti, pos, epoch, ws.hdr, ex, ok) && ok) {
                    double gagg[NX];
#pragma unroll
                    for (int c = 0; c < NX; ++c) gagg[c] = ex[c] + agg[c];
                    publish_pairs<NX>(ws.glb + (int64_t)g * kLbSlot, gagg,
                                      (epoch << 2) | kStateAgg);
                    (void)look_back_seq<NX>(ws.lb, ws.glb, ti, 0, g, epoch, ws.hdr, ex, lbs);
                }
            }
            SS_TRACE(ws, tile, 7);
            double inc[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) inc[c] = ex[c] + agg[c];
            publish_pairs<NX>(slot, inc, (epoch << 2) | kStateInc);
            if (leader)
                publish_pairs<NX>(ws.glb + (int64_t)g * kLbSlot, inc, (epoch << 2) | kStateInc);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < NX; ++c) s_excl[c] = ex[c];
            if constexpr (CARRY) {
                if (tile == ntiles - 1) {
                    s_fgw[0] = ex[Tx::EW] + agg[Tx::EW];
                    s_fgw[1] = ex[Tx::EXW] + agg[Tx::EXW];
                }
            }
        }
    }
    // the copy of G in LDS has landed: each wave waits for its own loads
    // (they count on its memory counter), the barrier for the others'
    if (g_lds) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    SS_TRACE(ws, tile, 3);
    // the products of step 5 are formed again below rather than kept live
    // across the look-back (registers bound how many tiles a CU holds)
    uint32_t xb = xbits;
    asm volatile("" : "+v"(xb));
    if (MODEL == SS_FINE_GRAY && !CARRY) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) asm volatile("" : "+v"(wv[i]));
    }
    if (MODEL == SS_FINE_GRAY && CARRY) {
        // w again (an L2 or last-level cache hit: the tile read it moments
        // ago) rather than held across the look-back: 28 fewer VGPRs at 16
        // positions per thread, three workgroups per CU instead of two
        // (measured 1721 -> 1649 us per coordinate at N = 2^27; without the
        // carried sums, held w measured faster, 1525 against 1600 us)
        const double *wsrc = a.w_comp;
        asm volatile("" : "+s"(wsrc));  // a new load, not the staged values
        if (cnt == TILE) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double2 *wp = reinterpret_cast<const double2 *>(
                    wsrc + t0 + (int64_t)q * BLOCK * C + (int64_t)tid * C);
#pragma unroll
                for (int h = 0; h < C / 2; ++h) {
                    const double2 v = wp[h];
                    wv[q * C + 2 * h] = v.x;
                    wv[q * C + 2 * h + 1] = v.y;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int64_t k = t0 + tile_pos<BLOCK, IPT>(i, tid);
                wv[i] = k < a.n ? wsrc[k] : 0.0;
            }
        }
    }
    // the tile's prefix: added to the FP64 in-tile prefixes now, or (F32S)
    // to each run end's FP32 in-tile prefix in FP64
    double carry[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) carry[c] = s_excl[c];
    if constexpr (!F32S) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < NX; ++c) texcl[q][c] += carry[c];
    }

    double tot[3] = {0.0, 0.0, 0.0};
    if (MODEL == SS_FINE_GRAY) {
#pragma unroll
        for (int c = 0; c < 3; ++c) tot[c] = ws.hdr->fg_tot[c];
    }

    // ---- 7. running prefix, transform at run ends, reduction
    asm volatile("" : "+v"(xb));
    AT acc_t[2] = {(AT)0, (AT)0};  // sum d G, sum d (H - G^2) of this thread
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    LogSum lsum;
    // Every event count of the wave's elements is 0 or 1 (and Fine-Gray
    // finds G in LDS): the run ends are evaluated without a branch, groups
    // of kTfGroup positions at a time so that their reciprocals overlap, and
    // a position without an event drops out through a select.  Measured at
    // N = 2^27 (IPT 16): Cox valued 580 -> 574 us, Fine-Gray with carried
    // totals 1417 -> 1354 us, but Cox 0/1 393 -> 400 us, which keeps the
    // branch.
    constexpr bool kFastTf = VALS || MODEL == SS_FINE_GRAY;
    bool small = true;
#pragma unroll
    for (int u = 0; u < (IPT + 3) / 4; ++u) small = small && (dw[u] & 0xfefefefeu) == 0u;
    const bool fast = kFastTf && __all(small) && (MODEL == SS_COX || g_lds);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        AT S[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) S[c] = texcl[q][c];
        if (fast) {
#pragma unroll
            for (int k0 = 0; k0 < C; k0 += kTfGroup) {
                double S0g[kTfGroup], S1g[kTfGroup], S2g[kTfGroup];
                bool evg[kTfGroup];
#pragma unroll
                for (int u = 0; u < kTfGroup; ++u) {
                    const int i = q * C + k0 + u;
                    const AT ei = (AT)ev[i];
                    Tx::add(S, ei, xb, i, s_xv, wv[MODEL == SS_FINE_GRAY ? i : 0]);
                    if constexpr (CARRY) {
                        const bool nb = (nbits >> i) & 1u;
                        const AT ew = ei * (AT)wv[i];
                        const bool xj = (xb >> i) & 1u;
                        acc[3] += nb ? (double)ew : 0.0;
                        acc[4] += nb && xj ? (double)ew : 0.0;
                    }
                    const bool ev1 = (dw[i / 4] >> (8 * (i % 4))) & 1u;
                    double Sd[NX];
#pragma unroll
                    for (int c = 0; c < NX; ++c)
                        Sd[c] = F32S ? carry[c] + (double)S[c] : (double)S[c];
                    double S0 = Sd[0], S1 = Sd[Tx::EX], S2 = Sd[Tx::EXX];
                    if (MODEL == SS_FINE_GRAY) {
                        const double gl =
                            s_g[w * (IPT * kWave) + (i / 2) * (2 * kWave) + 2 * lane + (i & 1)];
                        const double g = ev1 ? gl : 0.0;
                        S0 += g * (tot[0] - Sd[Tx::EW]);
                        S1 += g * (tot[1] - Sd[Tx::EXW]);
                        S2 = VALS ? S2 + g * (tot[2] - Sd[Tx::EXXW]) : S1;
                    }
                    S0g[u] = S0;
                    S1g[u] = S1;
                    S2g[u] = S2;
                    evg[u] = ev1;
                }
#pragma unroll
                for (int u = 0; u < kTfGroup; ++u) {
                    const AT r = recip((AT)S0g[u]);
                    const AT G = (AT)S1g[u] * r;
                    const AT H = VALS ? (AT)S2g[u] * r : G;
                    acc_t[0] += evg[u] ? G : (AT)0;
                    acc_t[1] += evg[u] ? H - G * G : (AT)0;
                    if (a.want_log) lsum.add01(S0g[u], evg[u] ? 1 : 0);
                }
            }
            lsum.renorm_all();
            continue;
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = q * C + k;
            const AT ei = (AT)ev[i];
            Tx::add(S, ei, xb, i, s_xv, wv[MODEL == SS_FINE_GRAY ? i : 0]);
            if constexpr (CARRY) {
                // sum e w and sum e w x_j over column jnext's positions
                const bool nb = (nbits >> i) & 1u;
                const AT ew = ei * (AT)wv[i];
                const bool xj = (xb >> i) & 1u;
                acc[3] += nb ? (double)ew : 0.0;
                acc[4] += nb && xj ? (double)ew : 0.0;
            }
            int d = (int)((dw[i / 4] >> (8 * (i % 4))) & 255u);
            if (d == 255) d = a.d32[t0 + tile_pos<BLOCK, IPT>(i, tid)];
            // the run end's prefix S0, S1, S2; Fine-Gray adds G(Y) times the
            // weighted suffix (the totals minus the inclusive prefix)
            double Sd[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) Sd[c] = F32S ? carry[c] + (double)S[c] : (double)S[c];
            double S0 = Sd[0], S1 = Sd[Tx::EX], S2 = Sd[Tx::EXX];
            if (MODEL == SS_FINE_GRAY) {
                double g = 0.0;
                if (d != 0) {
                    g = g_lds ? s_g[w * (IPT * kWave) + (i / 2) * (2 * kWave) + 2 * lane + (i & 1)]
                              : a.g_end[t0 + tile_pos<BLOCK, IPT>(i, tid)];
                }
                S0 += g * (tot[0] - Sd[Tx::EW]);
                S1 += g * (tot[1] - Sd[Tx::EXW]);
                S2 = VALS ? S2 + g * (tot[2] - Sd[Tx::EXXW]) : S1;
            }
            // (evaluating the transform at every position without a branch
            // holds far more registers)
            if (d != 0) {
                const AT r = recip((AT)S0);
                const AT G = (AT)S1 * r;
                const AT H = VALS ? (AT)S2 * r : G;
                const AT dd = (AT)d;
                acc_t[0] += dd * G;
                acc_t[1] += dd * (H - G * G);
                if (a.want_log) {
                    if (d > 1) lsum.add(S0, d);
                    else lsum.add01(S0, 1);
                }
            }
        }
        lsum.renorm_all();
    }
    acc[0] = (double)acc_t[0];
    acc[1] = (double)acc_t[1];
    if (a.want_log) acc[2] = lsum.value();
    block_sum<NR, BLOCK>(acc, s_red);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c) s_tsum[c] = acc[c];
    }
    __syncthreads();
    double tsum[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) tsum[c] = s_tsum[c];
    double total[NR];
    reduce_partials<BLOCK, NR, 8>(ws.part, ws.gpart, tile, ntiles, (epoch << 1) | 1u, ws.hdr,
                                  tsum, total, s_red);
    SS_TRACE(ws, tile, 4);
    if (tile == ntiles - 1) {
        finish<BLOCK, NR, CARRY>(a, ws, epoch, total, s_fgw, s_red);
        SS_TRACE(ws, tile, 5);
    }
}

// Fine-Gray totals pass: applies the pending step (a1) and reduces
// sum_r e_r x_r^m w_comp_r (m = 0, 1, 2) into hdr->fg_tot.
// With FP32 storage of e (ET = float) the sums are still FP64.
template <int BLOCK, int IPT, bool VALS, bool PREV, typename ET = double>
__global__ __launch_bounds__(BLOCK) void k_fg_totals(FusedCall a, WsView ws,
                                                     int64_t ntiles)
{
    constexpr int TILE = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ __attribute__((aligned(16))) uint8_t s_flag[TILE];
    __shared__ __attribute__((aligned(16))) double s_xv[VALS ? TILE : 1];
    __shared__ double s_ep[PREV ? TILE : 1];
    __shared__ double s_red[NW * 4];
    __shared__ double s_tsum[3];
    const int tid = threadIdx.x;
    // every wave reads the epoch itself (see k_fused)
    const uint64_t epoch = ld_relaxed_u64(&ws.hdr->fg_epoch);
    if (tid == 0 && a.clear_error && blockIdx.x == 0) st_relaxed_u32(&ws.hdr->error, 0u);
    clear_tile_lds<BLOCK, TILE, VALS>(s_flag, s_xv);
    __syncthreads();
    const uint64_t tag = (epoch << 1) | 1u;
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * TILE;
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = t0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + TILE / SS_CHUNK, nchunk);
    const int64_t cnt = min((int64_t)TILE, a.n - t0);
    ET ev[IPT];
    double wv[IPT];
    uint32_t dw[(IPT + 3) / 4];
    const uint32_t xbits = stage_tile<BLOCK, IPT, true, VALS, PREV, false, false, ET>(
        a, t0, cnt, chunk0, chunk1, s_flag, s_xv, s_ep, ev, wv, dw);
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const double x = x_at<BLOCK, VALS>(xbits, i, s_xv);
        const double ew = (double)ev[i] * wv[i];
        acc[0] += ew;
        acc[1] += ew * x;
        acc[2] += ew * x * x;
    }
    block_sum<3, BLOCK>(acc, s_red);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s_tsum[c] = acc[c];
    }
    __syncthreads();
    const double tsum[3] = {s_tsum[0], s_tsum[1], s_tsum[2]};
    double t[3];
    reduce_partials<BLOCK, 3, 4>(ws.fg_part, ws.fg_gpart, tile, ntiles, tag, ws.hdr, tsum, t,
                                 s_red);
    if (tile == ntiles - 1) {
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) ws.hdr->fg_tot[c] = t[c];
            st_relaxed_u64(&ws.hdr->fg_epoch, epoch + 1);
        }
    }
}

// a1 alone: eta += x step, e = exp(eta) at the non-zeros of column j.
template <bool VALS>
__global__ __launch_bounds__(256) void k_apply(int32_t j, const double *step,
                                               double *eta, double *e,
                                               const int64_t *col_ptr,
                                               const int32_t *rows,
                                               const double *vals)
{
    const double st = *step;
    if (st == 0.0) return;
    const int64_t cb = col_ptr[j];
    const int64_t nnz = col_ptr[j + 1] - cb;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nnz;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rows[cb + o];
        const double x = VALS ? vals[cb + o] : 1.0;
        const double et = eta[r] + x * st;
        eta[r] = et;
        e[r] = exp(et);
    }
}

__global__ void k_ccd_scalar(int penalty, double lambda, int32_t j,
                             const double *g12, double *beta, double *delta,
                             double *step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        ccd_apply(g12[0], g12[1], penalty, lambda, beta + j, delta + j, step);
}

__global__ void k_exp(int64_t n, const double *eta, double *e)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        e[i] = exp(eta[i]);
}

__global__ void k_gather(int64_t n, const int32_t *perm, const double *src,
                         double *dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[perm[i]];
}

__global__ void k_fill_zero(uint64_t *p, int64_t words)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

constexpr int kBlock = 256;

int grid_for(int64_t work, int per_block, int cap)
{
    int64_t g = ceil_div(work, per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

bool fused_ws_view(void *ws, size_t ws_bytes, int64_t n, WsView *v)
{
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < fused_ws_bytes(n)) return false;
    const int64_t tiles = ceil_div(n, SS_CHUNK) + 1;
    const int64_t groups = ceil_div(tiles, kGroup) + 1;
    char *p = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        u32x4 *r = (u32x4 *)(p + off);
        off = align_up(off + bytes, 256);
        return r;
    };
    v->hdr = (WsHeader *)p;
    off = sizeof(WsHeader);
    v->lb = take(16 * 8 * (size_t)tiles);
    v->glb = take(16 * 8 * (size_t)(ceil_div(tiles, kLbGroup) + 1));
    v->part = take(16 * 8 * (size_t)tiles);
    v->fg_part = take(16 * 4 * (size_t)tiles);
    v->gpart = take(16 * 8 * (size_t)groups);
    v->fg_gpart = take(16 * 4 * (size_t)groups);
    v->sw_agg = take(16 * 8 * (size_t)tiles);
    v->sw_part = take(16 * 4 * (size_t)tiles);
    v->sw_step = take(16 * (size_t)tiles);
    v->sw_pre = take(16 * 8 * (size_t)tiles);
    v->sw_pub = take(16 * (size_t)kSwPubWords);
    v->max_tiles = tiles;
    return true;
}

namespace {

template <int IPT, int MODEL, bool VALS, bool PREV, bool CARRY = false>
void launch_fused_t(const FusedCall &a, const WsView &ws, int64_t ntiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_fused<kBlock, IPT, MODEL, VALS, PREV, CARRY>), dim3((unsigned)ntiles),
                       dim3(kBlock), 0, s, a, ws, ntiles);
}

template <int IPT>
void launch_fg_totals_t(const FusedCall &a, const WsView &ws, int64_t ntiles, bool vals,
                        bool prev, hipStream_t s)
{
    const dim3 g((unsigned)ntiles), b(kBlock);
    if (vals) {
        if (prev) hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, true, true>), g, b, 0, s, a, ws, ntiles);
        else      hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, true, false>), g, b, 0, s, a, ws, ntiles);
    } else {
        if (prev) hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, false, true>), g, b, 0, s, a, ws, ntiles);
        else      hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, false, false>), g, b, 0, s, a, ws, ntiles);
    }
}

// FP32 storage of e: gradient and Hessian only (no pending update, no carry).
template <int IPT, int MODEL, bool VALS>
void launch_fused_f32_t(const FusedCall &a, const WsView &ws, int64_t ntiles, hipStream_t s)
{
    const dim3 g((unsigned)ntiles), b(kBlock);
    if (a.f32_sums)
        hipLaunchKernelGGL((k_fused<kBlock, IPT, MODEL, VALS, false, false, float, true>), g, b,
                           0, s, a, ws, ntiles);
    else
        hipLaunchKernelGGL((k_fused<kBlock, IPT, MODEL, VALS, false, false, float, false>), g,
                           b, 0, s, a, ws, ntiles);
}

template <int IPT>
int32_t launch_fused_f32_ipt(const FusedCall &a, const WsView &ws, int64_t ntiles,
                             hipStream_t s)
{
    const bool vals = a.col.vals != nullptr;
    if (a.jprev >= 0 || a.jnext >= 0 || a.ccd || a.fg_have_totals) return SS_EUNSUPPORTED;
    const dim3 g((unsigned)ntiles), b(kBlock);
    if (a.model == SS_FINE_GRAY) {
        if (vals) hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, true, false, float>), g, b, 0, s, a, ws, ntiles);
        else      hipLaunchKernelGGL((k_fg_totals<kBlock, IPT, false, false, float>), g, b, 0, s, a, ws, ntiles);
        SS_LAUNCH_CHECK();
        FusedCall c = a;
        c.clear_error = 0;
        if (vals) launch_fused_f32_t<IPT, SS_FINE_GRAY, true>(c, ws, ntiles, s);
        else      launch_fused_f32_t<IPT, SS_FINE_GRAY, false>(c, ws, ntiles, s);
    } else {
        if (vals) launch_fused_f32_t<IPT, SS_COX, true>(a, ws, ntiles, s);
        else      launch_fused_f32_t<IPT, SS_COX, false>(a, ws, ntiles, s);
    }
    SS_LAUNCH_CHECK();
    return SS_OK;
}

template <int IPT>
int32_t launch_fused_ipt(const FusedCall &a, const WsView &ws, hipStream_t s)
{
    const int64_t ntiles = ceil_div(a.n, (int64_t)kBlock * IPT);
    if (ntiles > ws.max_tiles) return SS_EWORKSPACE;
    if (a.e32) return launch_fused_f32_ipt<IPT>(a, ws, ntiles, s);
    const bool vals = a.col.vals != nullptr;
    const bool prev = a.jprev >= 0;
    FusedCall b = a;
    if (a.model == SS_FINE_GRAY) {
        // the carry of the weighted totals needs a 0/1 design
        const bool carry = a.jnext >= 0;
        if ((carry || a.fg_have_totals) && vals) return SS_EUNSUPPORTED;
        bool prev_scan = prev;
        if (!a.fg_have_totals) {
            // totals pass (and the pending a1 update), then the scan pass
            launch_fg_totals_t<IPT>(a, ws, ntiles, vals, prev, s);
            SS_LAUNCH_CHECK();
            b.jprev = -1;
            b.clear_error = 0;
            prev_scan = false;
        }
        if (vals) {
            launch_fused_t<IPT, SS_FINE_GRAY, true, false>(b, ws, ntiles, s);
        } else if (carry) {
            if (prev_scan) launch_fused_t<IPT, SS_FINE_GRAY, false, true, true>(b, ws, ntiles, s);
            else           launch_fused_t<IPT, SS_FINE_GRAY, false, false, true>(b, ws, ntiles, s);
        } else {
            if (prev_scan) launch_fused_t<IPT, SS_FINE_GRAY, false, true>(b, ws, ntiles, s);
            else           launch_fused_t<IPT, SS_FINE_GRAY, false, false>(b, ws, ntiles, s);
        }
    } else {
        if (vals) {
            if (prev) launch_fused_t<IPT, SS_COX, true, true>(b, ws, ntiles, s);
            else      launch_fused_t<IPT, SS_COX, true, false>(b, ws, ntiles, s);
        } else {
            if (prev) launch_fused_t<IPT, SS_COX, false, true>(b, ws, ntiles, s);
            else      launch_fused_t<IPT, SS_COX, false, false>(b, ws, ntiles, s);
        }
    }
    SS_LAUNCH_CHECK();
    return SS_OK;
}

// Gradient and Hessian, likelihood or objective alone (no pending update,
// no carry, no coordinate update): any tile shape.
template <int IPT>
int32_t launch_plain_ipt(const FusedCall &a, const WsView &ws, hipStream_t s)
{
    const int64_t ntiles = ceil_div(a.n, (int64_t)kBlock * IPT);
    if (ntiles > ws.max_tiles) return SS_EWORKSPACE;
    if (a.e32) return launch_fused_f32_ipt<IPT>(a, ws, ntiles, s);
    const bool vals = a.col.vals != nullptr;
    if (a.model == SS_FINE_GRAY) {
        launch_fg_totals_t<IPT>(a, ws, ntiles, vals, false, s);
        SS_LAUNCH_CHECK();
        FusedCall b = a;
        b.clear_error = 0;
        if (vals) launch_fused_t<IPT, SS_FINE_GRAY, true, false>(b, ws, ntiles, s);
        else      launch_fused_t<IPT, SS_FINE_GRAY, false, false>(b, ws, ntiles, s);
    } else {
        if (vals) launch_fused_t<IPT, SS_COX, true, false>(a, ws, ntiles, s);
        else      launch_fused_t<IPT, SS_COX, false, false>(a, ws, ntiles, s);
    }
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace

int32_t launch_fused(const FusedCall &a, const WsView &ws, hipStream_t s)
{
    const bool plain = a.jprev < 0 && a.jnext < 0 && !a.ccd && !a.fg_have_totals;
    if (plain) {
        const int32_t storage = !a.e32 ? SS_STORAGE_F64
                                : a.f32_sums ? SS_STORAGE_F32_SUMS32 : SS_STORAGE_F32;
        int32_t ipt = tune_lookup(SS_TUNE_GRAD_HESS, a.model, storage,
                                  a.col.vals != nullptr, a.n);
        if (!ipt) ipt = default_ipt(a.n);
        switch (ipt) {
        case 4: return launch_plain_ipt<4>(a, ws, s);
        case 8: return launch_plain_ipt<8>(a, ws, s);
        case 16: return launch_plain_ipt<16>(a, ws, s);
        case 32: return launch_plain_ipt<32>(a, ws, s);
        default: return SS_EINVAL;
        }
    }
    // the per-coordinate launches of a sweep (pending update, carry,
    // coordinate update): tiles of 2048 or 4096 positions
    if (a.e32) return SS_EUNSUPPORTED;
    return default_ipt(a.n) == 8 ? launch_fused_ipt<8>(a, ws, s) : launch_fused_ipt<16>(a, ws, s);
}

int32_t launch_apply(int64_t n, int32_t j, const double *step, double *eta,
                     double *e, const Column &col, hipStream_t s)
{
    const int grid = grid_for(n, 256, 2048);
    if (col.vals)
        hipLaunchKernelGGL(k_apply<true>, dim3(grid), dim3(256), 0, s, j, step, eta, e,
                           col.col_ptr, col.rows, col.vals);
    else
        hipLaunchKernelGGL(k_apply<false>, dim3(grid), dim3(256), 0, s, j, step, eta, e,
                           col.col_ptr, col.rows, col.vals);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_ccd_scalar(int32_t penalty, double lambda, int32_t j,
                          const double *g12, double *beta, double *delta,
                          double *step, hipStream_t s)
{
    hipLaunchKernelGGL(k_ccd_scalar, dim3(1), dim3(64), 0, s, penalty, lambda, j, g12,
                       beta, delta, step);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_exp(int64_t n, const double *eta, double *e, hipStream_t s)
{
    hipLaunchKernelGGL(k_exp, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, eta, e);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_gather(int64_t n, const int32_t *perm, const double *src,
                      double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, perm,
                       src, dst);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_ws_init(void *ws, size_t bytes, hipStream_t s)
{
    const int64_t words = (int64_t)(bytes / 8);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                       (uint64_t *)ws, words);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace ss
