// Persistent cyclic-coordinate-descent sweep for gfx950: the workflow of
// Fig. 3 (sparse update -> fused gradient/Hessian -> conditional update,
// for j = 1..P) in ONE cooperative launch, with no host round trip and no
// per-coordinate launch.
//
// Every workgroup owns a segment of S = BLOCK*IPT consecutive sorted
// positions for the whole sweep; e (and, for Fine-Gray, w and G) of its
// segment stay in registers, and only the rows that an update touches are
// patched.  Per coordinate j the workgroups exchange data twice:
//   1. all-to-one-to-all: each publishes the tuple aggregate of its
//      segment; workgroup 0 scans them in segment order and hands every
//      workgroup its exclusive prefix of the tuple scan (Sec. 2.7) -- and,
//      for Fine-Gray, the weighted suffix sum that starts at the segment
//      (eq. fg_g) -- a fixed-order computation, so results are
//      deterministic;
//   2. all-to-one-to-all: each publishes its partial sums of
//      d*G, d*(H - G^2), d*log S0; workgroup 0 adds them in order, takes the
//      coordinate update (Secs. 2.3-2.4) and broadcasts the step through one
//      flag per workgroup.
// Every exchanged value travels as a 16-byte (value, epoch tag) pair with
// one agent-scope access (no L2 flush or invalidate, no separate flag), so
// nothing is cleared between steps and O(segments) values move per
// exchange.
// Every wait is bounded; a timed-out wait sets the workspace error word and
// every workgroup leaves at its next wait.
#include "ss_device.h"

namespace ss {

namespace {

using namespace dev;

// Phase timestamps of the first 8 coordinates per workgroup, for
// performance-analysis builds only (-DSS_TRACE_TIMES).
#ifdef SS_TRACE_TIMES
#define SW_TRACE(a, b, jj, slot)                                                    \
    do {                                                                            \
        if (threadIdx.x == 0 && (jj) - (a).j_begin < 8)                             \
            trace_base((a).ws)                                                      \
                [((b) * 8 + ((jj) - (a).j_begin)) * 8 + (slot)] =                   \
                __builtin_amdgcn_s_memrealtime();                                   \
    } while (0)
#else
#define SW_TRACE(a, b, jj, slot) do { } while (0)
#endif

// Positions per group of the branch-free transform of k_sweep1.
#ifndef SS_SW_GROUP
#define SS_SW_GROUP 8
#endif
constexpr int kSwGroup = SS_SW_GROUP;
#ifndef SS_SW_FG_GROUP
#define SS_SW_FG_GROUP 4
#endif
constexpr int kSwFgGroup = SS_SW_FG_GROUP;  // the same for Fine-Gray

struct SweepArgs {
    int64_t n;
    int32_t j_begin;
    int32_t j_end;
    int32_t nblk;
    double *eta;
    double *e;
    const uint8_t *d8;
    const int32_t *d32;
    const double *w_comp;
    const double *g_end;
    Column col;
    const double *c;
    double *beta;
    double *delta;
    double *steps;
    double *g12_out;
    int32_t penalty;
    double lambda;
    int32_t want_log;
    WsView ws;
};

// Applies `st` times column jc to eta and e inside the segment; with LDS
// (s_ep, s_flag) also patches the registers of the owners.
template <int BLOCK, bool VALS, bool PATCH_LDS>
__device__ __forceinline__ void apply_step(const SweepArgs &a, int32_t jc, double st,
                                           int64_t seg0, int64_t chunk0, int64_t chunk1,
                                           double *s_ep, uint8_t *s_flag)
{
    const ColTile cp = col_tile(a.col, jc, chunk0, chunk1);
    for (int32_t o = cp.lo + (int32_t)threadIdx.x; o < cp.hi; o += BLOCK) {
        const int32_t k = a.col.rows[cp.cb + o];
        const double x = VALS ? a.col.vals[cp.cb + o] : 1.0;
        const double et = a.eta[k] + x * st;
        const double en = exp(et);
        a.eta[k] = et;
        a.e[k] = en;
        if (PATCH_LDS) {
            s_ep[k - seg0] = en;
            lds_flag_or(s_flag, (int32_t)(k - seg0), kFlagPatch);
        }
    }
}


template <int BLOCK, int IPT, int MODEL, bool VALS>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a)
{
    constexpr int S = BLOCK * IPT;
    constexpr bool FG = MODEL == SS_FINE_GRAY;
    constexpr int NC = FG ? 6 : 3;
    constexpr int NW = BLOCK / kWave;
    static_assert(S % SS_CHUNK == 0, "segment must be whole chunks");

    __shared__ __attribute__((aligned(16))) uint8_t s_flag[S];
    __shared__ double s_xv[VALS ? S : 1];
    __shared__ double s_ep[S];
    __shared__ double s_g[FG ? S : 1];
    __shared__ double s_wsum[NW][NC];
    __shared__ double s_wred[NW][3];
    __shared__ double s_bc[NC];
    __shared__ uint64_t s_ep0;
    __shared__ double s_step;
    __shared__ int s_abort;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t b = blockIdx.x;
    const int G = a.nblk;
    WsHeader *hdr = a.ws.hdr;
    const int64_t seg0 = b * S;
    const int64_t cnt = min((int64_t)S, a.n - seg0);
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = seg0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + S / SS_CHUNK, nchunk);
    const int64_t base = seg0 + (int64_t)tid * IPT;

    if (tid == 0) {
        s_ep0 = ld_relaxed_u64(&hdr->epoch);
        s_abort = 0;
    }

    // ---- the segment's data, kept for the whole sweep: e and w in
    // registers, G(y) in LDS (read only at the ends of event runs)
    double ev[IPT];
    int dk[IPT];
    double wv[FG ? IPT : 1];
    if (cnt == S) {
        const double2 *ep = reinterpret_cast<const double2 *>(a.e + base);
#pragma unroll
        for (int q = 0; q < IPT / 2; ++q) {
            const double2 v = ep[q];
            ev[2 * q] = v.x;
            ev[2 * q + 1] = v.y;
        }
        if (FG) {
            const double2 *wp = reinterpret_cast<const double2 *>(a.w_comp + base);
#pragma unroll
            for (int q = 0; q < IPT / 2; ++q) {
                const double2 v = wp[q];
                wv[2 * q] = v.x;
                wv[2 * q + 1] = v.y;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const bool ok = base + i < a.n;
            ev[i] = ok ? a.e[base + i] : 0.0;
            if (FG) wv[i] = ok ? a.w_comp[base + i] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t k = base + i;
        const bool ok = k < a.n;
        int d = ok ? (int)a.d8[k] : 0;
        if (d == 255) d = a.d32[k];
        dk[i] = d;
        if (FG) s_g[tid * IPT + i] = ok ? a.g_end[k] : 1.0;
    }
    __syncthreads();
    const uint64_t ep0 = s_ep0;

    for (int32_t j = a.j_begin; j < a.j_end; ++j) {
        const uint64_t ep = ep0 + (uint64_t)(j - a.j_begin);
        const uint64_t tag = (ep << 1) | 1u;
        SW_TRACE(a, b, j, 0);

        // ---- column j and the pending step of column j-1 into LDS
        {
            uint32_t *f32 = reinterpret_cast<uint32_t *>(s_flag);
            for (int i = tid; i < S / 4; i += BLOCK) f32[i] = 0u;
        }
        __syncthreads();
        {
            const ColTile cj = col_tile(a.col, j, chunk0, chunk1);
            for (int32_t o = cj.lo + tid; o < cj.hi; o += BLOCK) {
                const int32_t r = (int32_t)(a.col.rows[cj.cb + o] - seg0);
                if (VALS) s_xv[r] = a.col.vals[cj.cb + o];
                lds_flag_or(s_flag, r, kFlagX);
            }
        }
        if (j > a.j_begin) {
            if (tid == 0) {
                u32x4 r[1];
                if (wait_pairs<1>(a.ws.sw_step + b, ((ep - 1) << 1) | 1u, hdr, r))
                    s_step = pair_value(r[0]);
                else
                    s_abort = 1;
            }
            __syncthreads();
            SW_TRACE(a, b, j, 1);
            if (s_abort) return;
            const double st = s_step;
            if (st != 0.0)
                apply_step<BLOCK, VALS, true>(a, j - 1, st, seg0, chunk0, chunk1, s_ep, s_flag);
        }
        __syncthreads();
        SW_TRACE(a, b, j, 2);
        double xv[IPT];
        {
            uint8_t fl[IPT];
            lds_bytes<IPT>(s_flag + tid * IPT, fl);
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                if (VALS) xv[i] = (fl[i] & kFlagX) ? s_xv[tid * IPT + i] : 0.0;
                else xv[i] = (fl[i] & kFlagX) ? 1.0 : 0.0;
                if (fl[i] & kFlagPatch) ev[i] = s_ep[tid * IPT + i];
            }
        }

        // ---- thread totals, wave scans (DPP), segment aggregate
        double texcl[NC];
        {
            double run[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) run[c] = 0.0;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const double ex = ev[i] * xv[i];
                run[0] += ev[i];
                run[1] += ex;
                run[2] += ex * xv[i];
                if (FG) {
                    const double ew = ev[i] * wv[i];
                    const double exw = ew * xv[i];
                    run[3] += ew;
                    run[4] += exw;
                    run[5] += exw * xv[i];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double inc = dpp_incl_scan(run[c]);
                texcl[c] = inc - run[c];
                if (lane == kWave - 1) s_wsum[w][c] = inc;
            }
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) t += s_wsum[q][c];
                st_pair(a.ws.sw_agg + b * 8 + c, t, tag);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double before = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q)
                if (q < w) before += s_wsum[q][c];
            texcl[c] += before;
        }
        SW_TRACE(a, b, j, 3);

        // ---- exchange 1: workgroup 0 gathers every segment aggregate, scans
        // them in segment order and hands each workgroup its exclusive
        // prefix; for Fine-Gray the weighted components are handed over as
        // total minus exclusive prefix (the suffix sum that starts at the
        // segment).
        if (b == 0) {
            constexpr int K = (kMaxSweepBlocks + BLOCK - 1) / BLOCK;
            double v[K][NC];
            bool bad = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int q = tid * K + k;
#pragma unroll
                for (int c = 0; c < NC; ++c) v[k][c] = 0.0;
                if (q < G && !bad) {
                    u32x4 r[NC];
                    if (wait_pairs<NC>(a.ws.sw_agg + (int64_t)q * 8, tag, hdr, r)) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) v[k][c] = pair_value(r[c]);
                    } else {
                        bad = true;
                    }
                }
            }
            if (__syncthreads_or(bad)) return;
            // exclusive scan over q = tid*K + k: thread-serial, DPP across
            // lanes, LDS across waves
            double tsum[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) t += v[k][c];
                tsum[c] = t;
                const double inc = dpp_incl_scan(t);
                tsum[c] = inc - t;  // exclusive within the wave
                if (lane == kWave - 1) s_wsum[w][c] = inc;
            }
            __syncthreads();
            double tot3[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double before = 0.0, all = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    if (q < w) before += s_wsum[q][c];
                    all += s_wsum[q][c];
                }
                tsum[c] += before;
                if (FG && c >= 3) tot3[c - 3] = all;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int q = tid * K + k;
                if (q < G) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const double out = (FG && c >= 3) ? tot3[c - 3] - tsum[c] : tsum[c];
                        st_pair(a.ws.sw_pre + (int64_t)q * 8 + c, out, tag);
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) tsum[c] += v[k][c];
            }
        }
        if (tid == 0) {
            u32x4 r[NC];
            if (wait_pairs<NC>(a.ws.sw_pre + b * 8, tag, hdr, r)) {
#pragma unroll
                for (int c = 0; c < NC; ++c) s_bc[c] = pair_value(r[c]);
            } else {
                s_abort = 1;
            }
        }
        __syncthreads();
        SW_TRACE(a, b, j, 4);
        if (s_abort) return;

        // ---- running prefix, transform at run ends, reduction.  For
        // Fine-Gray R holds the weighted sums over the positions after the
        // current one (suffix sums, exclusive).
        double acc[3] = {0.0, 0.0, 0.0};
        {
            double Sr[3];
            double R[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; ++c) Sr[c] = texcl[c] + s_bc[c];
            if (FG) {
#pragma unroll
                for (int c = 0; c < 3; ++c) R[c] = s_bc[3 + c] - texcl[3 + c];
            }
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const double ex = ev[i] * xv[i];
                Sr[0] += ev[i];
                Sr[1] += ex;
                Sr[2] += ex * xv[i];
                if (FG) {
                    const double ew = ev[i] * wv[i];
                    const double exw = ew * xv[i];
                    R[0] -= ew;
                    R[1] -= exw;
                    R[2] -= exw * xv[i];
                }
                const int d = dk[i];
                if (d != 0) {
                    double S0 = Sr[0], S1 = Sr[1], S2 = Sr[2];
                    if (FG) {
                        const double g = s_g[tid * IPT + i];
                        S0 += g * R[0];
                        S1 += g * R[1];
                        S2 += g * R[2];
                    }
                    const double r = 1.0 / S0;
                    const double Gk = S1 * r;
                    const double Hk = S2 * r;
                    const double dd = (double)d;
                    acc[0] += dd * Gk;
                    acc[1] += dd * (Hk - Gk * Gk);
                    if (a.want_log) acc[2] += dd * log(S0);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] = dpp_wave_sum(acc[c]);
            if (lane == 0) s_wred[w][c] = acc[c];
        }
        __syncthreads();

        // ---- exchange 2: partials to workgroup 0, step back to everyone
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) t += s_wred[q][c];
                st_pair(a.ws.sw_part + b * 4 + c, t, tag);
            }
        }
        SW_TRACE(a, b, j, 5);
        if (b == 0) {
            constexpr int K = (kMaxSweepBlocks + BLOCK - 1) / BLOCK;
            double sum[3] = {0.0, 0.0, 0.0};
            bool bad = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int q = tid * K + k;
                if (q < G && !bad) {
                    u32x4 r[3];
                    if (wait_pairs<3>(a.ws.sw_part + (int64_t)q * 4, tag, hdr, r)) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) sum[c] += pair_value(r[c]);
                    } else {
                        bad = true;
                    }
                }
            }
            if (__syncthreads_or(bad)) return;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sum[c] = dpp_wave_sum(sum[c]);
                if (lane == 0) s_wred[w][c] = sum[c];
            }
            __syncthreads();
            if (tid == 0) {
                double tot[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int q = 0; q < NW; ++q) t += s_wred[q][c];
                    tot[c] = t;
                }
                const double g1 = a.c[j] - tot[0];
                const double g2 = -tot[1];
                double bj = a.beta[j], dj = a.delta[j], st = 0.0;
                ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &st);
                a.beta[j] = bj;
                a.delta[j] = dj;
                a.steps[j] = st;
                if (a.g12_out) {
                    a.g12_out[3 * j] = g1;
                    a.g12_out[3 * j + 1] = g2;
                    a.g12_out[3 * j + 2] = tot[2];
                }
                s_step = st;
            }
            __syncthreads();
            SW_TRACE(a, b, j, 6);
            const double st = s_step;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int q = tid * K + k;
                if (q < G) st_pair(a.ws.sw_step + q, st, tag);
            }
            SW_TRACE(a, b, j, 7);
        }
    }

    // ---- the last coordinate's update of eta and e
    const int32_t jl = a.j_end - 1;
    const uint64_t ep_last = ep0 + (uint64_t)(jl - a.j_begin);
    if (tid == 0) {
        u32x4 r[1];
        if (wait_pairs<1>(a.ws.sw_step + b, (ep_last << 1) | 1u, hdr, r))
            s_step = pair_value(r[0]);
        else
            s_abort = 1;
    }
    __syncthreads();
    if (s_abort) return;
    if (s_step != 0.0)
        apply_step<BLOCK, VALS, false>(a, jl, s_step, seg0, chunk0, chunk1, s_ep, s_flag);
    // every workgroup read the epoch before exchange 1 of the first
    // coordinate, which workgroup 0 waited for
    if (b == 0 && tid == 0)
        st_relaxed_u64(&hdr->epoch, ep0 + (uint64_t)(a.j_end - a.j_begin));
}

// ------------------------------------------------------------------------
// One exchange per coordinate, for 0/1 (indicator) designs.
//
// With x in {0, 1}, the update of column j multiplies e by exp(s_j) at the
// rows of column j, so a segment's tuple aggregate for the next coordinate
// is  A + expm1(s_j) D  with  A = sum e (1, x_{j+1})  over the segment and D
// the same sum over the rows of column j -- both known before s_j is.  Every
// workgroup therefore publishes, in one go, its partial sums for coordinate
// j together with A and D for coordinate j+1, then reads all G publications
// itself, forms the sums in the same fixed order, takes the same coordinate
// update (bit-identical everywhere) and its own prefix
// scan(A) + expm1(s_j) scan(D) over the segments before it.  (Gathering in
// workgroup 0 and broadcasting back was measured slower: 9.9 against 8.4 us
// per coordinate at N = 1e6, Cox.)
//
// Between its publication and the next coordinate's a workgroup touches
// global memory only for the exchange itself: e in registers, eta of its
// segment in LDS, the previous column patched in place (eta += s,
// e *= exp(s)), the rows of column j+2 scattered into LDS while the
// publications arrive.  Column c's rows live in bit (c mod 3) of the LDS
// flag bytes.  eta and e = exp(eta) go back to global memory once, at the
// end of the sweep.  Publications alternate between two slot sets by round parity:
// a workgroup can be at most one round ahead of the slowest reader (it
// needs everyone's publication of a round before it can publish the next),
// so a slot is never overwritten before all have read it.  c_j, beta_j and
// delta_j are read before publishing round j, and workgroup 0 writes beta_j
// and delta_j only after it has read every publication of that round, so
// no workgroup can see the updated values for the same coordinate.
template <int BLOCK, int IPT, int MODEL, bool LOG>
__global__ __launch_bounds__(BLOCK) void k_sweep1(SweepArgs a)
{
    constexpr int S = BLOCK * IPT;
    constexpr bool FG = MODEL == SS_FINE_GRAY;
    // With x in {0, 1}, e x^2 = e x: the tuple is (e, e x) for Cox and
    // (e, e x, e w, e w x) for Fine-Gray.
    constexpr int NT = FG ? 4 : 2;
    constexpr int NW = BLOCK / kWave;
    // partial sums: sum d G, sum d (G - G^2) and, with LOG, sum d log S0
    constexpr int P0 = LOG ? 3 : 2;
    constexpr int NPUB = P0 + 2 * NT;  // partial sums, A, D
    constexpr int NQ = pub_words<NPUB>();  // 16-byte words of a publication
    // Fine-Gray publications (8 words) go out in kPubCopies copies, one
    // word per lane of wave 0; the Cox ones (4-5 words) in one copy stored
    // by thread 0, which measured faster for them (5.88 against 5.92 ms per
    // 1000 coordinates at N = 1e6; Fine-Gray 11.5 -> 10.4 ms with copies)
    constexpr int NCOPY = FG ? kPubCopies : 1;
    static_assert(NQ <= kPubSlotWords && NQ * NCOPY <= kWave,
                  "one wave stores every copy of a publication");
    // block sums after a gather: partials (P0), A and D before this
    // segment (2 NT), and for Fine-Gray the totals of the weighted A and D
    // (4)
    constexpr int NSUM = P0 + 2 * NT + (FG ? 4 : 0);
    constexpr int K = (kMaxSweepBlocks + BLOCK - 1) / BLOCK;
    static_assert(K <= 2, "at most two segments per thread in a gather");
    static_assert(S % SS_CHUNK == 0, "segment must be whole chunks");

    __shared__ __attribute__((aligned(16))) uint8_t s_flag[S];
    __shared__ double s_eta[S];          // [i * BLOCK + tid]
    __shared__ double s_g[FG ? S : 1];   // G(y) at each position, same layout
    __shared__ double s_wsum[NW][NT];
    __shared__ double s_wred[NW][NPUB];
    __shared__ double s_sum[2][NW][NSUM];  // by round parity
    __shared__ uint64_t s_ep0;
    __shared__ int s_abort;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t b = blockIdx.x;
    const int G = a.nblk;
    WsHeader *hdr = a.ws.hdr;
    const int64_t seg0 = b * S;
    const int64_t cnt = min((int64_t)S, a.n - seg0);
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = seg0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + S / SS_CHUNK, nchunk);
    const int64_t base = seg0 + (int64_t)tid * IPT;
    const int32_t jb = a.j_begin, je = a.j_end;

    if (tid == 0) {
        s_ep0 = ld_relaxed_u64(&hdr->epoch);
        s_abort = 0;
    }
    // ---- the segment's data for the whole sweep
    double ev[IPT];
    int dk[IPT];
    double wv[FG ? IPT : 1];
    if (cnt == S) {
        const double2 *ep = reinterpret_cast<const double2 *>(a.e + base);
        const double2 *hp = reinterpret_cast<const double2 *>(a.eta + base);
#pragma unroll
        for (int q = 0; q < IPT / 2; ++q) {
            const double2 v = ep[q];
            const double2 h = hp[q];
            ev[2 * q] = v.x;
            ev[2 * q + 1] = v.y;
            s_eta[(2 * q) * BLOCK + tid] = h.x;
            s_eta[(2 * q + 1) * BLOCK + tid] = h.y;
        }
        if (FG) {
            const double2 *wp = reinterpret_cast<const double2 *>(a.w_comp + base);
#pragma unroll
            for (int q = 0; q < IPT / 2; ++q) {
                const double2 v = wp[q];
                wv[2 * q] = v.x;
                wv[2 * q + 1] = v.y;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const bool ok = base + i < a.n;
            ev[i] = ok ? a.e[base + i] : 0.0;
            s_eta[i * BLOCK + tid] = ok ? a.eta[base + i] : 0.0;
            if (FG) wv[i] = ok ? a.w_comp[base + i] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t k = base + i;
        const bool ok = k < a.n;
        int d = ok ? (int)a.d8[k] : 0;
        if (d == 255) d = a.d32[k];
        dk[i] = d;
        if (FG) s_g[i * BLOCK + tid] = ok ? a.g_end[k] : 1.0;
    }
    {
        uint32_t *f32 = reinterpret_cast<uint32_t *>(s_flag);
        for (int i = tid; i < S / 4; i += BLOCK) f32[i] = 0u;
    }
    __syncthreads();
    const uint64_t ep0 = s_ep0;

    // Adds column jc's rows of this segment as bit (jc mod 3), spread over
    // threads first .. BLOCK-1.
    auto scatter = [&](int32_t jc, int first) {
        const ColTile ct = col_tile(a.col, jc, chunk0, chunk1);
        const uint8_t bit = (uint8_t)(1u << (jc % 3));
        for (int32_t o = ct.lo + tid - first; o < ct.hi; o += BLOCK - first)
            lds_flag_or(s_flag, (int32_t)(a.col.rows[ct.cb + o] - seg0), bit);
    };
    // Clears bit (jc mod 3) in the bytes this thread owns.
    auto clear_bit = [&](int32_t jc) {
        const uint32_t keep = ~(0x01010101u << (jc % 3));
        uint32_t *f32 = reinterpret_cast<uint32_t *>(s_flag + tid * IPT);
#pragma unroll
        for (int q = 0; q < IPT / 4; ++q) f32[q] &= keep;
    };
    // Publication slot of segment q in round r, copy c: two sets by parity
    // inside each copy's area.  Workgroup b reads copy b mod NCOPY.
    auto pub_slot = [&](uint64_t r, int c, int64_t q) {
        return a.ws.sw_pub +
               (((int64_t)c * 2 + (r & 1u)) * kMaxSweepBlocks + q) * kPubSlotWords;
    };
    const int my_copy = (int)(b % NCOPY);
    // Block sums of NPUB values, published by wave 0 (Fine-Gray: lane l
    // stores word l mod NQ of copy l / NQ) or by thread 0 (Cox).
    auto publish = [&](double (&v)[NPUB], uint64_t r, uint64_t tag) {
#pragma unroll
        for (int c = 0; c < NPUB; ++c) {
            const double t = dpp_wave_sum(v[c]);
            if (lane == 0) s_wred[w][c] = t;
        }
        __syncthreads();
        if constexpr (!FG) {
            if (tid == 0) {
                u32x4 *dst = pub_slot(r, 0, b);
                double t[NPUB];
#pragma unroll
                for (int c = 0; c < NPUB; ++c) {
                    t[c] = 0.0;
#pragma unroll
                    for (int q = 0; q < NW; ++q) t[c] += s_wred[q][c];
                }
                u32x4 wd[NQ];
                pub_pack<NPUB>(t, (uint32_t)tag, wd);
#pragma unroll
                for (int c = 0; c < NQ; ++c) st_quad(dst + c, wd[c]);
            }
        } else if (w == 0) {
            double t[NPUB];
#pragma unroll
            for (int c = 0; c < NPUB; ++c) {
                t[c] = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) t[c] += s_wred[q][c];
            }
            u32x4 wd[NQ];
            pub_pack<NPUB>(t, (uint32_t)tag, wd);
            const int word = lane % NQ;
            // (an empty asm statement per word: a select chain over the
            // array itself is folded into an indexed load from scratch)
            u32x4 x = wd[0];
#pragma unroll
            for (int c = 1; c < NQ; ++c) {
                u32x4 y = wd[c];
                asm volatile("" : "+v"(y));
                x = word == c ? y : x;
            }
            if (lane < NQ * NCOPY) st_quad(pub_slot(r, lane / NQ, b) + word, x);
        }
    };
    // Reads every segment's publication of round r and forms the sums in a
    // fixed order (identical in every workgroup): out[0..2] partial sums,
    // out[3..] A and D over the segments before this one (then, for
    // Fine-Gray, the totals of the weighted A and D).  Returns false if a
    // wait gave up.
    auto gather = [&](uint64_t r, uint64_t tag, double (&out)[NSUM]) -> bool {
        double v[K][NPUB];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < NPUB; ++c) v[k][c] = 0.0;
        bool bad = false;
        const int q0 = tid * K;  // segments q0 .. q0 + K - 1
        if (K == 2 && q0 + 1 < G) {
            u32x4 r0[NQ], r1[NQ];
            uint32_t spins = 0;
            for (;;) {
                ld_pairs2<NQ>(pub_slot(r, my_copy, q0), r0, r1);
                if (pub_tagged<NQ>(r0, (uint32_t)tag) && pub_tagged<NQ>(r1, (uint32_t)tag))
                    break;
                if (((++spins & 31u) == 0 && ld_relaxed_u32(&hdr->error)) ||
                    spins > kSpinLimit) {
                    __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    bad = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (!bad) {
                pub_unpack<NPUB>(r0, v[0]);
                pub_unpack<NPUB>(r1, v[K - 1]);
            }
        } else if (q0 < G) {
            u32x4 rr[NQ];
            uint32_t spins = 0;
            for (;;) {
                ld_pairs<NQ>(pub_slot(r, my_copy, q0), rr);
                if (pub_tagged<NQ>(rr, (uint32_t)tag)) {
                    pub_unpack<NPUB>(rr, v[0]);
                    break;
                }
                if (((++spins & 31u) == 0 && ld_relaxed_u32(&hdr->error)) ||
                    spins > kSpinLimit) {
                    __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    bad = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        double t[NSUM];
#pragma unroll
        for (int c = 0; c < NSUM; ++c) t[c] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool before = q0 + k < b;
#pragma unroll
            for (int c = 0; c < P0; ++c) t[c] += v[k][c];
#pragma unroll
            for (int c = 0; c < 2 * NT; ++c) t[P0 + c] += before ? v[k][P0 + c] : 0.0;
            if (FG) {
                // weighted components of A (indices 2, 3) and D (2, 3), all segments
                t[P0 + 2 * NT + 0] += v[k][P0 + 2];
                t[P0 + 2 * NT + 1] += v[k][P0 + 3];
                t[P0 + 2 * NT + 2] += v[k][P0 + NT + 2];
                t[P0 + 2 * NT + 3] += v[k][P0 + NT + 3];
            }
        }
        const int par = (int)(r & 1u);
#pragma unroll
        for (int c = 0; c < NSUM; ++c) {
            const double x = dpp_wave_sum(t[c]);
            if (lane == 0) s_sum[par][w][c] = x;
        }
        if (__syncthreads_or(bad)) return false;
#pragma unroll
        for (int c = 0; c < NSUM; ++c) {
            double x = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) x += s_sum[par][q][c];
            out[c] = x;
        }
        return true;
    };
    // prefix of this segment (Fine-Gray: plus the suffix starts) for the
    // coordinate after an update s, from the gathered sums
    auto prefix_from = [&](const double (&sm)[NSUM], double st, double (&pre)[NT]) {
        const double f = expm1(st);
#pragma unroll
        for (int c = 0; c < NT; ++c) pre[c] = sm[P0 + c] + f * sm[P0 + NT + c];
        if (FG) {
#pragma unroll
            for (int c = 2; c < 4; ++c) {
                const double tot = sm[P0 + 2 * NT + (c - 2)] + f * sm[P0 + 2 * NT + 2 + (c - 2)];
                pre[c] = tot - pre[c];
            }
        }
    };

    // ---- round 0: aggregates of coordinate jb; rows of jb and jb+1
    scatter(jb, 0);
    if (jb + 1 < je) scatter(jb + 1, 0);
    __syncthreads();
    double pre[NT];
    {
        double v[NPUB];
#pragma unroll
        for (int c = 0; c < NPUB; ++c) v[c] = 0.0;
        uint8_t fl[IPT];
        lds_bytes<IPT>(s_flag + tid * IPT, fl);
        const uint8_t bj = (uint8_t)(1u << (jb % 3));
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            v[P0] += ev[i];
            v[P0 + 1] += (fl[i] & bj) ? ev[i] : 0.0;
            if (FG) {
                const double ew = ev[i] * wv[i];
                v[P0 + 2] += ew;
                v[P0 + 3] += (fl[i] & bj) ? ew : 0.0;
            }
        }
        const uint64_t tag = (ep0 << 1) | 1u;
        publish(v, 0, tag);
        double sm[NSUM];
        if (!gather(0, tag, sm)) return;
        prefix_from(sm, 0.0, pre);
    }
    double st_prev = 0.0;

    for (int32_t j = jb; j < je; ++j) {
        const uint64_t r = (uint64_t)(j - jb) + 1;  // exchange round of coordinate j
        const uint64_t tag = ((ep0 + r) << 1) | 1u;
        SW_TRACE(a, b, j, 0);
        // the coordinate's constants, read before this round is published
        const double cj = a.c[j];
        double bj = a.beta[j], dj = a.delta[j];
        uint8_t fl[IPT];
        lds_bytes<IPT>(s_flag + tid * IPT, fl);
        const uint8_t bcur = (uint8_t)(1u << (j % 3));
        const uint8_t bnext = (uint8_t)(1u << ((j + 1) % 3));
        const uint8_t bprev = (uint8_t)(1u << ((j + 2) % 3));
        // ---- the update of column j-1, in place
        if (j > jb && st_prev != 0.0) {
            const double fe = exp(st_prev);
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                if (fl[i] & bprev) {
                    // LDS atomic add, result unused: no wait for a read
                    // (only this thread touches the position, in order)
                    __hip_atomic_fetch_add(&s_eta[i * BLOCK + tid], st_prev, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    ev[i] *= fe;
                }
            }
        }
        SW_TRACE(a, b, j, 1);
        // ---- in-segment scan of the tuple of coordinate j
        double texcl[NT];
        double run[NT];  // thread totals, also the A and D of j+1 that sum all e
        {
#pragma unroll
            for (int c = 0; c < NT; ++c) run[c] = 0.0;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                run[0] += ev[i];
                run[1] += (fl[i] & bcur) ? ev[i] : 0.0;
                if (FG) {
                    const double ew = ev[i] * wv[i];
                    run[2] += ew;
                    run[3] += (fl[i] & bcur) ? ew : 0.0;
                }
            }
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const double inc = dpp_incl_scan(run[c]);
                texcl[c] = inc - run[c];
                if (lane == kWave - 1) s_wsum[w][c] = inc;
            }
        }
        __syncthreads();
        // every thread has read its flags: column j-1's bit is free
        clear_bit(j + 2);
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            double before = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q)
                if (q < w) before += s_wsum[q][c];
            texcl[c] += before;
        }
        SW_TRACE(a, b, j, 2);
        // ---- transform and reduction of coordinate j; A and D of j+1
        double v[NPUB];
#pragma unroll
        for (int c = 0; c < NPUB; ++c) v[c] = 0.0;
        {
            double Sr[2], R[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 2; ++c) Sr[c] = pre[c] + texcl[c];
            if (FG) {
#pragma unroll
                for (int c = 0; c < 2; ++c) R[c] = pre[2 + c] - texcl[2 + c];
            }
            const bool has_next = j + 1 < je;
            // S0 and S1 at a group of positions first, then the transform
            // at all of them at once, masked by the event count: the
            // reciprocals are independent and overlap (one wave per SIMD
            // here, nothing else hides their latency; run by run behind a
            // branch each one waited for the last: Cox 8.08 -> 7.22 ms per
            // 1000 coordinates at N = 1e6).  Fine-Gray, which holds far more
            // registers, groups kSwFgGroup positions (10.32 -> 10.20 ms at
            // 4; with an IEEE division instead of the reciprocal, grouping
            // 8 had measured 12.8 -> 13.0 ms).
            constexpr int GT = FG ? kSwFgGroup : (IPT < kSwGroup ? IPT : kSwGroup);
#pragma unroll
            for (int i0 = 0; i0 < IPT; i0 += GT) {
                double s0v[GT], s1v[GT];
#pragma unroll
                for (int u = 0; u < GT; ++u) {
                    const int i = i0 + u;
                    const bool xc = fl[i] & bcur;
                    const bool xn = has_next && (fl[i] & bnext);
                    const double ex = xc ? ev[i] : 0.0;
                    Sr[0] += ev[i];
                    Sr[1] += ex;
                    double ew = 0.0, ewx = 0.0;
                    if (FG) {
                        ew = ev[i] * wv[i];
                        ewx = xc ? ew : 0.0;
                        R[0] -= ew;
                        R[1] -= ewx;
                    }
                    double S0 = Sr[0], S1 = Sr[1];
                    if (FG) {
                        const double g = s_g[i * BLOCK + tid];
                        S0 += g * R[0];
                        S1 += g * R[1];
                    }
                    s0v[u] = S0;
                    s1v[u] = S1;
                    // A (all positions) and D (rows of column j) for j+1 on
                    // the rows of column j+1; the sums over all positions
                    // are the thread totals of the scan (same terms, same
                    // order)
                    v[P0 + 1] += xn ? ev[i] : 0.0;
                    v[P0 + 1 + NT] += xn ? ex : 0.0;
                    if (FG) {
                        v[P0 + 3] += xn ? ew : 0.0;
                        v[P0 + 3 + NT] += xn ? ewx : 0.0;
                    }
                }
                // indicator design: S2 = S1, so H = G; S0 > 0 everywhere (it
                // holds e of the position itself or of one before it)
                if constexpr (FG && GT > 1) {
#pragma unroll
                    for (int u = 0; u < GT; ++u) {
                        const double Gk = s1v[u] * recip(s0v[u]);
                        const double dd = (double)dk[i0 + u];  // 0 off the run ends
                        v[0] = fma(dd, Gk, v[0]);
                        v[1] = fma(dd, Gk - Gk * Gk, v[1]);
                    }
                    if constexpr (LOG) {
#pragma unroll
                        for (int u = 0; u < GT; ++u)
                            if (dk[i0 + u] != 0) v[2] += (double)dk[i0 + u] * log(s0v[u]);
                    }
                } else if constexpr (FG) {
                    const int d = dk[i0];
                    if (d != 0) {
                        // hardware estimate and Newton steps, as Cox (an
                        // IEEE division measured 10.46 against 10.34 ms
                        // per 1000 coordinates at N = 1e6)
                        const double Gk = s1v[0] * recip(s0v[0]);
                        const double dd = (double)d;
                        v[0] += dd * Gk;
                        v[1] += dd * (Gk - Gk * Gk);
                        if constexpr (LOG) v[2] += dd * log(s0v[0]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < GT; ++u) {
                        const double Gk = s1v[u] * recip(s0v[u]);
                        const double dd = (double)dk[i0 + u];  // 0 off the run ends
                        v[0] = fma(dd, Gk, v[0]);
                        v[1] = fma(dd, Gk - Gk * Gk, v[1]);
                    }
                    if constexpr (LOG) {
#pragma unroll
                        for (int u = 0; u < GT; ++u)
                            if (dk[i0 + u] != 0) v[2] += (double)dk[i0 + u] * log(s0v[u]);
                    }
                }
            }
            v[P0] = run[0];
            v[P0 + NT] = run[1];
            if (FG) {
                v[P0 + 2] = run[2];
                v[P0 + 2 + NT] = run[3];
            }
        }
        publish(v, r, tag);
        SW_TRACE(a, b, j, 3);
        // ---- rows of column j+2 while the publications arrive
        if (j + 2 < je) scatter(j + 2, 0);
        // ---- every segment's publication: the update of j, the prefix of j+1
        double sm[NSUM];
        if (!gather(r, tag, sm)) return;
        SW_TRACE(a, b, j, 4);
        double st = 0.0;
        {
            const double g1 = cj - sm[0];
            const double g2 = -sm[1];
            ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &st);
            if (b == 0 && tid == 0) {
                a.beta[j] = bj;
                a.delta[j] = dj;
                a.steps[j] = st;
                if (a.g12_out) {
                    a.g12_out[3 * j] = g1;
                    a.g12_out[3 * j + 1] = g2;
                    a.g12_out[3 * j + 2] = LOG ? sm[2] : 0.0;
                }
            }
        }
        prefix_from(sm, st, pre);
        st_prev = st;
        SW_TRACE(a, b, j, 5);
    }

    // ---- the last coordinate's update, then eta and e back to memory
    {
        uint8_t fl[IPT];
        lds_bytes<IPT>(s_flag + tid * IPT, fl);
        const uint8_t blast = (uint8_t)(1u << ((je - 1) % 3));
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int64_t k = base + i;
            if (k < a.n) {
                double h = s_eta[i * BLOCK + tid];
                if (st_prev != 0.0 && (fl[i] & blast)) h += st_prev;
                a.eta[k] = h;
                a.e[k] = exp(h);
            }
        }
    }
    // every workgroup read the epoch before publishing round 0, which
    // workgroup 0 has gathered
    if (b == 0 && tid == 0)
        st_relaxed_u64(&hdr->epoch, ep0 + (uint64_t)(je - jb) + 1);
}

// Shapes tried in order: the first whose workgroups all fit on the device at
// once (a cooperative launch requires it) is used.
struct Shape {
    int block;
    int ipt;
};

template <int BLOCK, int IPT, int MODEL, bool VALS>
void *kernel_ptr()
{
    return reinterpret_cast<void *>(&k_sweep<BLOCK, IPT, MODEL, VALS>);
}

template <int BLOCK, int IPT, int MODEL>
void *kernel1_ptr(bool log)
{
    return log ? reinterpret_cast<void *>(&k_sweep1<BLOCK, IPT, MODEL, true>)
               : reinterpret_cast<void *>(&k_sweep1<BLOCK, IPT, MODEL, false>);
}

// Indicator designs take the one-exchange kernel, valued ones the general.
// (the one-exchange kernel publishes sum d log S0 only when it is asked for)
template <int BLOCK, int IPT>
void *pick_kernel(int model, bool vals, bool log)
{
    if (model == SS_FINE_GRAY)
        return vals ? kernel_ptr<BLOCK, IPT, SS_FINE_GRAY, true>()
                    : kernel1_ptr<BLOCK, IPT, SS_FINE_GRAY>(log);
    return vals ? kernel_ptr<BLOCK, IPT, SS_COX, true>() : kernel1_ptr<BLOCK, IPT, SS_COX>(log);
}

void *kernel_for(int block, int ipt, int model, bool vals, bool log)
{
    if (block == 256 && ipt == 8) return pick_kernel<256, 8>(model, vals, log);
    if (block == 256 && ipt == 16) return pick_kernel<256, 16>(model, vals, log);
    if (block == 512 && ipt == 8) return pick_kernel<512, 8>(model, vals, log);
    // 8192-position segments: Cox only (Fine-Gray would not fit its LDS or
    // would spill registers)
    if (block == 512 && ipt == 16 && model == SS_COX)
        return vals ? kernel_ptr<512, 16, SS_COX, true>() : kernel1_ptr<512, 16, SS_COX>(log);
    return nullptr;
}

}  // namespace

int32_t launch_sweep_persistent(const SweepCall &call, const WsView &ws, hipStream_t s)
{
    // segments of 2048 to 8192 positions; LDS holds a segment's flags,
    // column values, patched e and (Fine-Gray) G(y)
    static const Shape shapes_valued[] = {{256, 8}, {256, 16}, {512, 8}, {512, 16}};
    // 0/1 designs: every workgroup reads all G publications per coordinate;
    // 256 x 16 measured fastest (N = 1e6, Cox: 8.5 us per coordinate against
    // 11.8 us at 512 x 16, where two waves share each SIMD)
    static const Shape shapes_01[] = {{256, 16}, {512, 8}, {256, 8}, {512, 16}};
    int dev = 0;
    SS_HIP_CHECK(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    SS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SS_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return SS_EUNSUPPORTED;
    const bool vals = call.col.vals != nullptr;
    // a tuned shape first, then the built-in order; a shape forced by a
    // tuning call alone
    Shape order[5];
    int m = 0;
    const int32_t want = tune_lookup(SS_TUNE_SWEEP, call.model, SS_STORAGE_F64, vals, call.n);
    if (want) order[m++] = Shape{want / 100, want % 100};
    if (!(tune_force().choice && tune_force().kind == SS_TUNE_SWEEP)) {
        for (const Shape &sh : vals ? shapes_valued : shapes_01)
            if (sh.block * 100 + sh.ipt != want) order[m++] = sh;
    }
    for (int o = 0; o < m; ++o) {
        const Shape &sh = order[o];
        const int64_t seg = (int64_t)sh.block * sh.ipt;
        const int64_t G = ceil_div(call.n, seg);
        // a few hundred segments at most: the all-to-all exchange reads G
        // aggregates per workgroup
        if (G > kMaxSweepBlocks || G > ws.max_tiles) continue;
        void *k = kernel_for(sh.block, sh.ipt, call.model, vals, call.g12_out != nullptr);
        if (!k) continue;
        int per_cu = 0;
        SS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, sh.block, 0));
        if ((int64_t)per_cu * cus < G) continue;
        SweepArgs a;
        a.n = call.n;
        a.j_begin = call.j_begin;
        a.j_end = call.j_end;
        a.nblk = (int32_t)G;
        a.eta = call.eta;
        a.e = call.e;
        a.d8 = call.d8;
        a.d32 = call.d32;
        a.w_comp = call.w_comp;
        a.g_end = call.g_end;
        a.col = call.col;
        a.c = call.c;
        a.beta = call.beta;
        a.delta = call.delta;
        a.steps = call.steps;
        a.g12_out = call.g12_out;
        a.penalty = call.penalty;
        a.lambda = call.lambda;
        a.want_log = call.g12_out != nullptr;
        a.ws = ws;
        void *args[] = {&a};
        SS_HIP_CHECK(hipLaunchCooperativeKernel(k, dim3((unsigned)G), dim3((unsigned)sh.block),
                                                args, 0, s));
        return SS_OK;
    }
    return SS_EUNSUPPORTED;
}

}  // namespace ss
