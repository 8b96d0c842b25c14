// Cross-validation replicates in one launch (Sec. 2.8; the single larger
// kernel for many repetitions of k-fold cross-validation that the paper's
// concluding discussion proposes in place of one stream per fold).
//
// All replicates share the subjects' order by decreasing time, the tie runs
// and the design X; each has its own training mask, linear predictor eta,
// coefficients and trust-region widths.  A replicate is the data set of its
// training subjects: its held-out subjects carry e = 0, so they drop out of
// every prefix sum, and its event counts per run end and its c_j count
// training events only.  eta is kept for every subject (X beta), so the
// held-out log-likelihood can be evaluated at the fitted beta.
//
// One workgroup of 1024 threads runs one replicate's coordinates in order:
// the scan of coordinate j goes over the replicate in chunks of 1024 x IPT
// positions (each thread owns the same IPT consecutive positions of every
// chunk for the whole launch), the thread sums are combined by one wave scan
// and one barrier per chunk, the transform and reduction follow in
// registers, and the Newton step of Sec. 2.4 is taken by thread 0.  No
// workgroup ever waits for another, so the launch needs no co-residency, and
// the summation order is fixed (deterministic results).
//
// Designs with x in {0, 1} (the Sec. 3.2 designs): column j is read as a
// dense bitmask (stride/8 bytes per column, one load per thread per chunk)
// instead of row indices, the update of column j multiplies e by exp(s) in
// place at its rows, and S2 = S1 since x^2 = x.  e is recomputed as exp(eta)
// when the launch ends.
#include <math.h>
#include <stdlib.h>

#include "ss_device.h"

namespace ss {

namespace {

using namespace dev;

constexpr int kCvBlock = 1024;
constexpr int kCvWaves = kCvBlock / kWave;
constexpr int kCvAlign = 16384;  // per-replicate stride unit (a whole chunk)
constexpr int kCvList = 512;
#ifndef SS_CV_FG_BLOCK
#define SS_CV_FG_BLOCK 512
#endif
#ifndef SS_CV_FG_IPT
#define SS_CV_FG_IPT 8
#endif
#ifndef SS_CV_COX_BLOCK
#define SS_CV_COX_BLOCK 1024
#endif
constexpr int kCvFgBlock = SS_CV_FG_BLOCK;
constexpr int kCvCoxBlock = SS_CV_COX_BLOCK;
constexpr int kCvFgIpt = SS_CV_FG_IPT;     // non-zero steps held before eta is brought up to date
constexpr int kCvGather = 16;    // column bitmask loads in flight while eta is updated
// share of a replicate's chunks taken by half 0 of a two-half launch
// (measured at N = 1e5 .. 4e5, 100 replicates: 12/25 against 2/5, 5/11
// and 1/2)
constexpr int kCvSplitNum = 12;
constexpr int kCvSplitDen = 25;

__device__ __forceinline__ bool cv_event(int32_t model, int8_t s)
{
    return model == SS_FINE_GRAY ? s == 1 : s != 0;
}

// Prefix over the 16 wave totals of a chunk: lane q < 16 holds wave q's
// total; an inclusive scan within the first DPP row of 16 lanes, then the
// calling wave takes the sum of the waves before it and the chunk total.
template <int NW = kCvWaves>
__device__ __forceinline__ void wave_totals_prefix(double v, int w, double &before,
                                                   double &total)
{
    static_assert(NW <= 16, "one DPP row");
    v += dpp_double<0x111, 0xF, true>(v);  // row_shr:1
    v += dpp_double<0x112, 0xF, true>(v);  // row_shr:2
    v += dpp_double<0x114, 0xF, true>(v);  // row_shr:4
    v += dpp_double<0x118, 0xF, true>(v);  // row_shr:8
    total = read_lane(v, NW - 1);
    before = w > 0 ? read_lane(v, w - 1) : 0.0;
}

__device__ __forceinline__ uint64_t lanes_below(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

// ---------------------------------------------------------------- prepare
// Per replicate, in sorted order: the training flag, the training events
// per run end (the run's events among the training subjects, at the
// position where the full data set has its run end with events), and the
// training-event bitmask (for c_j).  A run end with events is where the
// full data set's count is non-zero; runs without events there hold no
// training events either, so the training events of a run are the
// training events after the previous such position.
__global__ __launch_bounds__(kCvBlock) void k_cv_prep(int32_t model, int64_t n, int64_t stride,
                                                      const int32_t *perm, const int8_t *status,
                                                      const uint8_t *train, const uint8_t *d8,
                                                      uint8_t *train_s, uint8_t *d8_r,
                                                      int32_t *d32_r, uint32_t *evbits)
{
    __shared__ int s_cnt[kCvWaves];
    __shared__ int s_last[kCvWaves];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t r = blockIdx.x;
    const uint8_t *tr_in = train + r * n;
    const int64_t off = r * stride;
    int carry_cnt = 0;   // training events before the chunk
    int carry_last = 0;  // their count at the last run end with events
    for (int64_t base = 0; base < stride; base += kCvBlock) {
        const int64_t k = base + tid;
        int tr = 0, ev = 0, mark = 0;
        if (k < n) {
            const int32_t i = perm[k];
            tr = tr_in[i] != 0;
            ev = tr && cv_event(model, status[i]);
            mark = d8[k] != 0;
        }
        const uint64_t bev = __ballot(ev);
        const uint64_t bmark = __ballot(mark);
        const int cnt_w = __popcll(bev & (lanes_below(lane) | (1ull << lane)));
        if (lane == kWave - 1) s_cnt[w] = __popcll(bev);
        __syncthreads();
        int before = carry_cnt, total = carry_cnt;
        for (int q = 0; q < kCvWaves; ++q) {
            const int v = s_cnt[q];
            if (q < w) before += v;
            total += v;
        }
        const int cnt = before + cnt_w;  // inclusive count at k
        // count at the nearest run end with events in this wave, below k
        const uint64_t below = bmark & lanes_below(lane);
        const int src = below ? 63 - __clzll(below) : lane;
        const int v_below = __shfl(cnt, src);
        const int v_top = __shfl(cnt, bmark ? 63 - __clzll(bmark) : 0);
        if (lane == 0) s_last[w] = bmark ? v_top : -1;
        __syncthreads();
        int prev = carry_last, last = carry_last;
        for (int q = 0; q < kCvWaves; ++q) {
            const int v = s_last[q];
            if (v >= 0) {
                if (q < w) prev = v;
                last = v;
            }
        }
        if (below) prev = v_below;
        const int d = mark ? cnt - prev : 0;
        train_s[off + k] = (uint8_t)tr;
        d8_r[off + k] = (uint8_t)(d >= 255 ? 255 : d);
        if (d >= 255) d32_r[off + k] = d;
        if (lane == 0) evbits[(off + k) / 32] = (uint32_t)bev;
        if (lane == 32) evbits[(off + k) / 32] = (uint32_t)(bev >> 32);
        carry_cnt = total;
        carry_last = last;
        __syncthreads();
    }
}


// Kaplan-Meier estimates of the censoring distribution per replicate, for
// the Fine-Gray weights of Sec. 2.2 (reading: G(t) = prod over censoring
// times c <= t of (1 - m_c / n_c), right-continuous): one for the training
// subjects (the replicate's own data set) and one for the held-out subjects
// (the data set its held-out likelihood is scored on).  In sorted order
// (decreasing time) G at position k is the product of one factor per tie
// run from k's run to the end: m_c / n_c are the run's censored subjects of
// the subset and the subset's subjects at or before the run's end.  Pass 1
// writes the factors at run ends (1 elsewhere), pass 2 turns them into the
// suffix product (last chunk first; thread t takes the chunk's position
// 1023 - t, so a prefix product over the threads is a suffix product over
// the positions).  Outputs per replicate: g_r = G of the training subset and
// g_h = G of the held-out subset at every position, w_r = I(training and
// status 2) / g_r; the stride's padding gets G = 1, w = 0.
__device__ __forceinline__ double wave_incl_prod(double x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double y = __shfl_up(x, d);
        if (lane >= d) x *= y;
    }
    return x;
}

__global__ __launch_bounds__(kCvBlock) void k_cv_km(int64_t n, int64_t stride,
                                                    const int32_t *perm, const int8_t *status,
                                                    const double *y, const uint8_t *train_s,
                                                    double *w_r, double *g_r, double *g_h)
{
    __shared__ int s_cnt[4][kCvWaves];
    __shared__ int s_last[2][kCvWaves];
    __shared__ double s_prod[2][kCvWaves];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t r = blockIdx.x;
    const int64_t off = r * stride;
    // pass 1: the factor of every tie run at its last position
    int carry[4] = {0, 0, 0, 0};  // subset sizes and censored counts before the chunk
    int carry_last[2] = {0, 0};   // censored counts at the last run end before it
    for (int64_t base = 0; base < n; base += kCvBlock) {
        const int64_t k = base + tid;
        bool flag[4] = {false, false, false, false};  // train, train cens, held, held cens
        bool re = false;
        if (k < n) {
            const bool tr = train_s[off + k] != 0;
            const int8_t st = status[perm[k]];
            flag[0] = tr;
            flag[1] = tr && st == 0;
            flag[2] = !tr;
            flag[3] = !tr && st == 0;
            re = k == n - 1 || y[perm[k + 1]] != y[perm[k]];
        }
        int cnt[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t b = __ballot(flag[q]);
            cnt[q] = __popcll(b & (lanes_below(lane) | (1ull << lane)));
            if (lane == kWave - 1) s_cnt[q][w] = __popcll(b);
        }
        const uint64_t bre = __ballot(re);
        __syncthreads();
        int tot[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int before = carry[q];
            tot[q] = carry[q];
            for (int v = 0; v < kCvWaves; ++v) {
                const int c = s_cnt[q][v];
                if (v < w) before += c;
                tot[q] += c;
            }
            cnt[q] += before;  // inclusive count at k
        }
        // censored counts at the nearest run end below k
        const uint64_t below = bre & lanes_below(lane);
        const int src = below ? 63 - __clzll(below) : lane;
        const int top = bre ? 63 - __clzll(bre) : 0;
        int prevc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cc = cnt[2 * h + 1];
            const int v_below = __shfl(cc, src);
            const int v_top = __shfl(cc, top);
            if (lane == 0) s_last[h][w] = bre ? v_top : -1;
            prevc[h] = v_below;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int prev = carry_last[h], last = carry_last[h];
            for (int v = 0; v < kCvWaves; ++v) {
                const int c = s_last[h][v];
                if (c >= 0) {
                    if (v < w) prev = c;
                    last = c;
                }
            }
            if (below) prev = prevc[h];
            double f = 1.0;
            if (re) {
                const int m = cnt[2 * h + 1] - prev;
                const int at = cnt[2 * h];
                if (m > 0) f = 1.0 - (double)m / (double)at;
            }
            if (k < n) (h == 0 ? g_r : g_h)[off + k] = f;
            carry_last[h] = last;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) carry[q] = tot[q];
        __syncthreads();
    }
    // pass 2: suffix products, last chunk first
    double carry_p[2] = {1.0, 1.0};
    const int64_t nch = (n + kCvBlock - 1) / kCvBlock;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        const int64_t k = ch * kCvBlock + (kCvBlock - 1 - tid);
        double f[2] = {1.0, 1.0};
        if (k < n) {
            f[0] = g_r[off + k];
            f[1] = g_h[off + k];
        }
        double inc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            inc[h] = wave_incl_prod(f[h]);
            if (lane == kWave - 1) s_prod[h][w] = inc[h];
        }
        __syncthreads();
        double G[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double before = carry_p[h], all = carry_p[h];
            for (int v = 0; v < kCvWaves; ++v) {
                const double q = s_prod[h][v];
                if (v < w) before *= q;
                all *= q;
            }
            G[h] = before * inc[h];
            carry_p[h] = all;
        }
        if (k < n) {
            const bool tr = train_s[off + k] != 0;
            g_r[off + k] = G[0];
            g_h[off + k] = G[1];
            w_r[off + k] = tr && status[perm[k]] == 2 ? 1.0 / G[0] : 0.0;
        }
        __syncthreads();
    }
    for (int64_t k = n + tid; k < stride; k += kCvBlock) {
        g_r[off + k] = 1.0;
        g_h[off + k] = 1.0;
        w_r[off + k] = 0.0;
    }
}

// Column bitmask of a 0/1 design: bit k of column j is set where x_kj = 1
// (k a sorted position).  The mask is cleared beforehand.
__global__ __launch_bounds__(256) void k_cv_bits(int64_t p, int64_t words,
                                                 const int64_t *col_ptr,
                                                 const int32_t *rows_sorted, uint32_t *xbits)
{
    for (int64_t j = blockIdx.x; j < p; j += gridDim.x) {
        const int64_t lo = col_ptr[j], hi = col_ptr[j + 1];
        for (int64_t q = lo + threadIdx.x; q < hi; q += 256) {
            const int32_t k = rows_sorted[q];
            atomicOr(&xbits[j * words + (k >> 5)], 1u << (k & 31));
        }
    }
}

// c_j of every replicate: the training events with x_kj = 1.
// Fine-Gray: bit k of the extra column p is set where the subject at
// sorted position k had a competing event (status 2).  The mask is cleared
// beforehand.
__global__ __launch_bounds__(256) void k_cv_comp_bits(int64_t n, const int32_t *perm,
                                                      const int8_t *status, uint32_t *bits)
{
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        const uint64_t b = __ballot(status[perm[k]] == 2);
        // lanes 0 and 32 of the wave write their 32-position words
        const int lane = lane_id();
        if ((lane & 31) == 0 && (k & 31) == 0) bits[k >> 5] = (uint32_t)(b >> lane);
    }
}

__global__ __launch_bounds__(256) void k_cv_c(int64_t p, int64_t words, const uint32_t *xbits,
                                              const uint32_t *evbits, double *c)
{
    __shared__ int s_red[4];
    const int64_t j = blockIdx.x;
    const int64_t r = blockIdx.y;
    const uint32_t *xb = xbits + j * words;
    const uint32_t *eb = evbits + r * words;
    int cnt = 0;
    for (int64_t q = threadIdx.x; q < words; q += 256) cnt += __popc(xb[q] & eb[q]);
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) c[r * p + j] = (double)(s_red[0] + s_red[1] + s_red[2] + s_red[3]);
}

__global__ __launch_bounds__(256) void k_cv_exp(int64_t total, const double *eta,
                                                const uint8_t *train_s, double *e)
{
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256)
        e[k] = train_s[k] ? exp(eta[k]) : 0.0;
}

__global__ __launch_bounds__(256) void k_cv_fill(uint32_t *p, int64_t words)
{
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < words; k += (int64_t)gridDim.x * 256)
        p[k] = 0u;
}

// ---------------------------------------------------------------- sweep
// Exchange block of one replicate (two-half launches): the epoch of its
// exchanges, then per round parity a slot of half 0 and one of half 1, each
// a run of 16-byte (value, tag) pairs.
constexpr int kCvXchBytes = 1280;

struct CvArgs {
    int64_t n, p, stride;
    int64_t j_begin, j_end;
    int32_t reps;
    int32_t penalty;
    double lambda;
    double *eta, *e;
    const uint8_t *d8;
    const int32_t *d32;
    const uint8_t *train_s;
    const uint8_t *xbits;
    const double *c;
    double *beta, *delta, *g12_out;
    WsHeader *hdr;  // the sticky error word of bounded waits
    char *xch;      // exchange blocks, kCvXchBytes per replicate
};

__device__ __forceinline__ uint64_t *cv_epoch(const CvArgs &a, int64_t r)
{
    return reinterpret_cast<uint64_t *>(a.xch + r * kCvXchBytes);
}

__device__ __forceinline__ u32x4 *cv_slot(const CvArgs &a, int64_t r, int h, int par)
{
    return reinterpret_cast<u32x4 *>(a.xch + r * kCvXchBytes + 256 + (par * 2 + h) * 256);
}

template <int IPT>
struct CvChunk {
    double v[IPT];
    uint32_t d[IPT / 4];  // event counts, one byte per position
    uint32_t x;           // column j at the thread's positions
    uint32_t px;          // the pending column
    uint32_t x1;          // column j + 1 (half 0 of a two-half launch)
};

template <int IPT>
__device__ __forceinline__ uint32_t cv_bits(const CvArgs &a, int64_t j, int64_t pos)
{
    static_assert(IPT == 8 || IPT == 16, "whole bytes of the column bitmask per thread");
    const uint8_t *col = a.xbits + j * (a.stride / 8) + pos / 8;
    if constexpr (IPT == 16) return *reinterpret_cast<const uint16_t *>(col);
    else return *col;
}

template <int IPT>
__device__ __forceinline__ void cv_load(const CvArgs &a, const double *e, const uint8_t *d8,
                                        int64_t pos, int64_t j, int64_t jp, int64_t j1,
                                        CvChunk<IPT> &c)
{
    const double2 *src = reinterpret_cast<const double2 *>(e + pos);
#pragma unroll
    for (int i = 0; i < IPT / 2; ++i) {
        const double2 t = src[i];
        c.v[2 * i] = t.x;
        c.v[2 * i + 1] = t.y;
    }
    if constexpr (IPT == 16) {
        const uint4 q = *reinterpret_cast<const uint4 *>(d8 + pos);
        c.d[0] = q.x; c.d[1] = q.y; c.d[2] = q.z; c.d[3] = q.w;
    } else {
        const uint2 q = *reinterpret_cast<const uint2 *>(d8 + pos);
        c.d[0] = q.x; c.d[1] = q.y;
    }
    c.x = cv_bits<IPT>(a, j, pos);
    c.px = jp >= 0 ? cv_bits<IPT>(a, jp, pos) : 0u;
    c.x1 = j1 >= 0 ? cv_bits<IPT>(a, j1, pos) : 0u;
}

// eta += step * x_j at this thread's positions of chunks [ch_lo, ch_hi)
// for the listed steps, in the order they were taken (the order a
// coordinate-by-coordinate update would add them); with `resync`,
// e = exp(eta) at training positions and 0 elsewhere afterwards.  Column
// bitmasks are fetched kCvGather at a time.
template <int IPT, int BLOCK = kCvBlock>
__device__ void cv_apply_steps(const CvArgs &a, double *eta, double *e, const uint8_t *train_s,
                               const int32_t *lj, const double *ls, int nlist, int ch_lo,
                               int ch_hi, int64_t tpos, bool resync)
{
    constexpr int CHUNK = BLOCK * IPT;
    for (int ch = ch_lo; ch < ch_hi; ++ch) {
        const int64_t pos = (int64_t)ch * CHUNK + tpos;
        double v[IPT];
        const double2 *src = reinterpret_cast<const double2 *>(eta + pos);
#pragma unroll
        for (int i = 0; i < IPT / 2; ++i) {
            const double2 t = src[i];
            v[2 * i] = t.x;
            v[2 * i + 1] = t.y;
        }
        for (int q0 = 0; q0 < nlist; q0 += kCvGather) {
            uint32_t b[kCvGather];
#pragma unroll
            for (int u = 0; u < kCvGather; ++u)
                b[u] = q0 + u < nlist ? cv_bits<IPT>(a, lj[q0 + u], pos) : 0u;
#pragma unroll
            for (int u = 0; u < kCvGather; ++u) {
                if (b[u] != 0u) {
                    const double st = ls[q0 + u];
#pragma unroll
                    for (int i = 0; i < IPT; ++i)
                        if ((b[u] >> i) & 1u) v[i] += st;
                }
            }
        }
        double2 *dst = reinterpret_cast<double2 *>(eta + pos);
#pragma unroll
        for (int i = 0; i < IPT / 2; ++i) dst[i] = make_double2(v[2 * i], v[2 * i + 1]);
        if (resync) {
            double2 *ed = reinterpret_cast<double2 *>(e + pos);
#pragma unroll
            for (int i = 0; i < IPT / 2; ++i)
                ed[i] = make_double2(train_s[pos + 2 * i] ? exp(v[2 * i]) : 0.0,
                                     train_s[pos + 2 * i + 1] ? exp(v[2 * i + 1]) : 0.0);
        }
    }
}

// KH = 1: one workgroup per replicate.  KH = 2: two, each holding half of
// the replicate's chunks (a cooperative launch, so both are resident).  Per
// coordinate the halves exchange once: half 1 publishes its partial sums;
// half 0 publishes its partial sums, c_j, beta_j, delta_j and what half 1
// needs for its carry of the NEXT coordinate.  With x in {0, 1} the step s
// multiplies e by exp(s) at column j, so half 0's totals for coordinate
// j + 1 are A0 + expm1(s) D0 (all e; D0 = e at column j) and
// A1 + expm1(s) D1 (e at column j + 1; D1 = e at both columns), all
// summed during the pass of coordinate j before s is known.  Both halves
// then take the same Newton step from the same numbers.
template <int BLOCK, int IPT, int KH>
__global__ __launch_bounds__(BLOCK) void k_cv_sweep(CvArgs a)
{
    constexpr int CHUNK = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ double s_tot[2][NW][2];
    __shared__ double s_red[NW * 4];
    __shared__ double s_step[4];  // step, exp(step), half 1's next carry
    __shared__ int32_t s_lj[kCvList];
    __shared__ double s_ls[kCvList];
    __shared__ int s_ln;
    __shared__ int s_abort;
    __shared__ uint64_t s_ep0;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    int64_t r;
    int h;
    if constexpr (KH == 1) {
        r = blockIdx.x;
        h = 0;
    } else {
        // the two halves of a replicate are 8 workgroups apart, which puts
        // them on the same XCD (workgroups go round-robin over the 8)
        const int b = (int)blockIdx.x;
        r = (int64_t)(b / 16) * 8 + (b % 8);
        h = (b % 16) / 8;
        if (r >= a.reps) return;
    }
    const int64_t off = r * a.stride;
    double *eta = a.eta + off;
    double *e = a.e + off;
    const uint8_t *d8 = a.d8 + off;
    const int32_t *d32 = a.d32 + off;
    // chunks that hold subjects (the stride's padding beyond n is skipped;
    // its e stays 0)
    const int nch = (int)min(a.stride / CHUNK, (a.n + CHUNK - 1) / CHUNK);
    // half 0 also sums what half 1's next carry needs, so it takes fewer
    // of the chunks: kCvSplitNum / kCvSplitDen of them, rounded
    const int chm = (nch * kCvSplitNum + kCvSplitDen / 2) / kCvSplitDen;
    const int ch_lo = (KH == 2 && h == 1) ? chm : 0;
    const int ch_hi = (KH == 2 && h == 0) ? chm : nch;
    const int64_t tpos = (int64_t)tid * IPT;
    const bool lead = h == 0;                 // owns beta, delta, g12_out
    const bool sums_next = KH == 2 && h == 0;  // sums for half 1's next carry
    const int64_t T = a.j_end - a.j_begin;

    if (tid == 0) {
        s_ln = 0;
        s_abort = 0;
        s_ep0 = KH == 2 ? ld_relaxed_u64(cv_epoch(a, r)) : 0;
    }
    __syncthreads();
    const uint64_t ep0 = s_ep0;
    double k0 = 0.0, k1 = 0.0;  // half 1: half 0's totals of the coordinate

    // round 0 of a two-half launch: half 1's carry for the first coordinate
    if (KH == 2 && T > 0) {
        const uint64_t tag = (ep0 << 1) | 1u;
        if (h == 0) {
            double x[2] = {0.0, 0.0};
            for (int ch = ch_lo; ch < ch_hi; ++ch) {
                const int64_t pos = (int64_t)ch * CHUNK + tpos;
                const double2 *src = reinterpret_cast<const double2 *>(e + pos);
                const uint32_t xb = cv_bits<IPT>(a, a.j_begin, pos);
#pragma unroll
                for (int i = 0; i < IPT / 2; ++i) {
                    const double2 t = src[i];
                    x[0] += t.x + t.y;
                    x[1] += (((xb >> (2 * i)) & 1u) ? t.x : 0.0) +
                            (((xb >> (2 * i + 1)) & 1u) ? t.y : 0.0);
                }
            }
            block_sum<2, BLOCK>(x, s_red);
            if (tid == 0) {
                u32x4 *sl = cv_slot(a, r, 0, 0);
                st_pair(sl + 0, x[0], tag);
                st_pair(sl + 1, x[1], tag);
                st_pair(sl + 2, 0.0, tag);
            }
        } else {
            if (tid == 0) {
                u32x4 rr[3];
                if (wait_pairs<3>(cv_slot(a, r, 0, 0), tag, a.hdr, rr)) {
                    s_step[2] = pair_value(rr[0]);
                    s_step[3] = pair_value(rr[1]);
                } else {
                    s_abort = 1;
                    s_step[2] = s_step[3] = 0.0;
                }
            }
            __syncthreads();
            k0 = s_step[2];
            k1 = s_step[3];
        }
    }

    double s_prev = 0.0, es_prev = 1.0;  // the pending step and exp of it
    int64_t jp = -1;                     // its column
    CvChunk<IPT> cur;
    const bool any = ch_lo < ch_hi;
    if (T > 0 && any)
        cv_load<IPT>(a, e, d8, (int64_t)ch_lo * CHUNK + tpos, a.j_begin, -1,
                     sums_next && a.j_begin + 1 < a.j_end ? a.j_begin + 1 : -1, cur);
    int par = 0;
    for (int64_t j = a.j_begin; j < a.j_end && !s_abort; ++j) {
        // the lead's thread 0 fetches what the update needs now, uses it at
        // the end
        double cj = 0.0, bj = 0.0, dj = 0.0;
        if (lead && tid == 0) {
            cj = a.c[r * a.p + j];
            bj = a.beta[r * a.p + j];
            dj = a.delta[r * a.p + j];
        }
        double acc1 = 0.0, acc2 = 0.0, a1 = 0.0, d1 = 0.0;
        double carry0 = k0, carry1 = k1;
        for (int ch = ch_lo; ch < ch_hi; ++ch) {
            const int64_t pos = (int64_t)ch * CHUNK + tpos;
            // a1: the pending step of column jp at this thread's positions
            // (e only: eta is brought up to date from the list of steps)
            if (cur.px != 0u && s_prev != 0.0) {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if ((cur.px >> i) & 1u) cur.v[i] *= es_prev;
                double2 *dst = reinterpret_cast<double2 *>(e + pos);
#pragma unroll
                for (int i = 0; i < IPT / 2; ++i)
                    dst[i] = make_double2(cur.v[2 * i], cur.v[2 * i + 1]);
            }
            // event counts; runs of 255 or more events read their count
            // now, before the prefetch below, so that waiting for these
            // rare loads never waits for the prefetch (loads complete in
            // order)
            uint32_t dv[IPT];
#pragma unroll
            for (int i = 0; i < IPT; ++i) dv[i] = (cur.d[i / 4] >> (8 * (i % 4))) & 0xffu;
#pragma unroll
            for (int i = 0; i < IPT; ++i)
                if (dv[i] == 255u) dv[i] = (uint32_t)d32[pos + i];
            // the next chunk (of this coordinate or the next) is in flight
            // during this one's arithmetic; issued after the stores above,
            // which it may read when there is a single chunk.  After the
            // last coordinate it re-reads column j (unused), so the number
            // of loads in flight is the same on every path.
            CvChunk<IPT> nx;
            const bool last = ch + 1 == ch_hi;
            const int64_t jn = last ? (j + 1 < a.j_end ? j + 1 : j) : j;
            const int64_t jn1 = sums_next && jn + 1 < a.j_end ? jn + 1 : -1;
            cv_load<IPT>(a, e, d8, last ? (int64_t)ch_lo * CHUNK + tpos : pos + CHUNK, jn,
                         last ? j : jp, jn1, nx);

            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                t0 += cur.v[i];
                t1 += ((cur.x >> i) & 1u) ? cur.v[i] : 0.0;
            }
            if (sums_next) {
                const uint32_t both = cur.x & cur.x1;
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    a1 += ((cur.x1 >> i) & 1u) ? cur.v[i] : 0.0;
                    d1 += ((both >> i) & 1u) ? cur.v[i] : 0.0;
                }
            }
            const double i0 = dpp_incl_scan(t0);
            const double i1 = dpp_incl_scan(t1);
            if (lane == kWave - 1) {
                s_tot[par][w][0] = i0;
                s_tot[par][w][1] = i1;
            }
            __syncthreads();
            double b0, b1, T0, T1;
            wave_totals_prefix<NW>(lane < NW ? s_tot[par][lane][0] : 0.0, w, b0, T0);
            wave_totals_prefix<NW>(lane < NW ? s_tot[par][lane][1] : 0.0, w, b1, T1);
            const double p0 = carry0 + b0, p1 = carry1 + b1;
            const double c0 = carry0 + T0, c1 = carry1 + T1;
            par ^= 1;
            double S0 = p0 + (i0 - t0);
            double S1 = p1 + (i1 - t1);
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                S0 += cur.v[i];
                S1 += ((cur.x >> i) & 1u) ? cur.v[i] : 0.0;
                const uint32_t d = dv[i];
                if (d != 0u) {
                    const double g = S1 / S0;
                    const double dd = (double)d;
                    acc1 = fma(dd, g, acc1);
                    acc2 = fma(dd, g - g * g, acc2);
                }
            }
            carry0 = c0;
            carry1 = c1;
            cur = nx;
        }
        // g' = c_j - sum d S1/S0, g'' = -sum d (S2/S0 - (S1/S0)^2), S2 = S1
        double red[4] = {acc1, acc2, a1, d1};
        if (sums_next) block_sum<4, BLOCK>(red, s_red);
        else block_sum<2, BLOCK>(*reinterpret_cast<double(*)[2]>(red), s_red);
        if (tid == 0) {
            double g1, g2, step = 0.0;
            bool ok = true;
            if constexpr (KH == 2) {
                const int64_t t = j - a.j_begin + 1;
                const uint64_t tag = ((ep0 + (uint64_t)t) << 1) | 1u;
                const int q = (int)(t & 1);
                double h0[9], h1[2];
                if (h == 0) {
                    h0[0] = red[0]; h0[1] = red[1];
                    h0[2] = carry0; h0[3] = carry1;  // A0, D0
                    h0[4] = red[2]; h0[5] = red[3];  // A1, D1
                    h0[6] = cj; h0[7] = bj; h0[8] = dj;
                    u32x4 *sl = cv_slot(a, r, 0, q);
#pragma unroll
                    for (int m = 0; m < 9; ++m) st_pair(sl + m, h0[m], tag);
                    u32x4 rr[3];
                    ok = wait_pairs<3>(cv_slot(a, r, 1, q), tag, a.hdr, rr);
                    h1[0] = pair_value(rr[0]);
                    h1[1] = pair_value(rr[1]);
                } else {
                    h1[0] = red[0]; h1[1] = red[1];
                    u32x4 *sl = cv_slot(a, r, 1, q);
                    st_pair(sl + 0, h1[0], tag);
                    st_pair(sl + 1, h1[1], tag);
                    st_pair(sl + 2, 0.0, tag);
                    u32x4 rr[9];
                    ok = wait_pairs<9>(cv_slot(a, r, 0, q), tag, a.hdr, rr);
#pragma unroll
                    for (int m = 0; m < 9; ++m) h0[m] = pair_value(rr[m]);
                    cj = h0[6]; bj = h0[7]; dj = h0[8];
                }
                g1 = cj - (h0[0] + h1[0]);
                g2 = -(h0[1] + h1[1]);
                if (ok) ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &step);
                if (h == 1) {
                    const double em = expm1(step);
                    s_step[2] = fma(em, h0[3], h0[2]);
                    s_step[3] = fma(em, h0[5], h0[4]);
                }
            } else {
                g1 = cj - red[0];
                g2 = -red[1];
                ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &step);
            }
            if (!ok) s_abort = 1;
            if (lead && ok) {
                a.beta[r * a.p + j] = bj;
                a.delta[r * a.p + j] = dj;
                if (a.g12_out) {
                    double *o = a.g12_out + (r * a.p + j) * 3;
                    o[0] = g1;
                    o[1] = g2;
                    o[2] = step;
                }
            }
            s_step[0] = step;
            s_step[1] = exp(step);
            if (step != 0.0) {
                s_lj[s_ln] = (int32_t)j;
                s_ls[s_ln] = step;
                s_ln = s_ln + 1;
            }
        }
        __syncthreads();
        s_prev = s_step[0];
        es_prev = s_step[1];
        if (KH == 2 && h == 1) {
            k0 = s_step[2];
            k1 = s_step[3];
        }
        jp = j;
        if (s_ln == kCvList) {  // uniform: every thread reads the same count
            cv_apply_steps<IPT, BLOCK>(a, eta, e, a.train_s + off, s_lj, s_ls, kCvList, ch_lo, ch_hi,
                                tpos, false);
            __syncthreads();
            if (tid == 0) s_ln = 0;
            __syncthreads();
        }
    }

    // eta brought up to date, and e = exp(eta) afresh (masked) everywhere
    cv_apply_steps<IPT, BLOCK>(a, eta, e, a.train_s + off, s_lj, s_ls, s_ln, ch_lo, ch_hi, tpos, true);
    // half 0 has seen half 1's last publication, made after half 1 read the
    // epoch: the next launch's tags start after this launch's
    if (KH == 2 && h == 0 && tid == 0 && T > 0 && !s_abort)
        st_relaxed_u64(cv_epoch(a, r), ep0 + (uint64_t)T + 1);
}


// ---------------------------------------------------------------- Fine-Gray
// Fine-Gray model, 0/1 design.  The tuple of Sec. 2.7 has four distinct
// components here (e, e x, e w, e x w; x^2 = x), and each run end with
// training events needs, besides the prefix sums, G of the replicate's
// training subset times the weighted suffix: the totals T = sum e w and
// Tx = sum e w x_j of the replicate minus the inclusive prefixes of e w and
// e x w.  The totals are needed before the scan, so they are carried from
// one coordinate to the next in closed form: the step s of column j
// multiplies e by exp(s) at its rows, so the totals of column j + 1 are
// A + expm1(s) D and A1 + expm1(s) D1, with A = sum e w, D = sum e w x_j,
// A1 = sum e w x_{j+1}, D1 = sum e w x_j x_{j+1} summed during the pass of
// column j.  A pass before the first coordinate sums the totals of column
// j_begin.  w = 1/G where the subject had a competing event (a bit column
// after the design's columns), 0 elsewhere: the division the preparation
// makes for w_r, so the same bits.
//
// KH = 2: two workgroups per replicate, the halves of its chunks, as in the
// Cox sweep.  Half 1 starts each coordinate from half 0's sums of the four
// components, which half 0 gives it in closed form from the previous pass
// (its sums of e, e x_j, e w, e w x_j and of e x_{j+1}, e x_j x_{j+1},
// e w x_{j+1}, e w x_j x_{j+1}); before the first coordinate half 1 sums
// them itself over half 0's chunks.  Per coordinate the halves exchange once
// (half 0: its partial sums, those eight, c_j, beta_j, delta_j; half 1: its
// partial sums, its prefix carries of e w and e w x_j, which end as the
// replicate's, and its sums for A1, D1) and both take the same step and the
// same next totals from the same numbers.  Summation order fixed
// (deterministic).
struct CvFgArgs {
    CvArgs a;
    const double *g;  // g_r: G of the training subset
};

// w at a thread's IPT positions from G and the competing-event bits.
template <int IPT>
__device__ __forceinline__ void fg_weights(uint32_t cb, const double (&gv)[IPT],
                                           double (&wv)[IPT])
{
#pragma unroll
    for (int i = 0; i < IPT; ++i) wv[i] = ((cb >> i) & 1u) && gv[i] != 0.0 ? 1.0 / gv[i] : 0.0;
}

template <int IPT>
__device__ __forceinline__ void fg_load_g(const double *gr, int64_t pos, double (&gv)[IPT])
{
    const double2 *gs = reinterpret_cast<const double2 *>(gr + pos);
#pragma unroll
    for (int i = 0; i < IPT / 2; ++i) {
        const double2 u = gs[i];
        gv[2 * i] = u.x;
        gv[2 * i + 1] = u.y;
    }
}

// Sums over chunks [lo, hi) of e, e x_j, e w, e w x_j (the four components
// of column j), in the workgroup's fixed order; every thread gets them.
template <int BLOCK, int IPT>
__device__ void fg_sums(const CvArgs &a, const double *e, const double *gr, int64_t j, int lo,
                        int hi, int64_t tpos, double *s_red, double *s_bc, double (&out)[4])
{
    constexpr int CHUNK = BLOCK * IPT;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    for (int ch = lo; ch < hi; ++ch) {
        const int64_t pos = (int64_t)ch * CHUNK + tpos;
        const uint32_t xb = cv_bits<IPT>(a, j, pos);
        double gv[IPT], wv[IPT];
        fg_load_g<IPT>(gr, pos, gv);
        fg_weights<IPT>(cv_bits<IPT>(a, a.p, pos), gv, wv);
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const double ev = e[pos + i];
            const double ew = ev * wv[i];
            const bool xi = (xb >> i) & 1u;
            x[0] += ev;
            x[1] += xi ? ev : 0.0;
            x[2] += ew;
            x[3] += xi ? ew : 0.0;
        }
    }
    block_sum<4, BLOCK>(x, s_red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s_bc[c] = x[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = s_bc[c];
    __syncthreads();
}

template <int BLOCK, int IPT, int KH>
__global__ __launch_bounds__(BLOCK) void k_cv_sweep_fg(CvFgArgs f)
{
    const CvArgs &a = f.a;
    constexpr int CHUNK = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ double s_tot[2][NW][4];
    __shared__ double s_red[NW * 6];
    // step, exp(step), the next column's totals, half 1's next carries
    __shared__ double s_step[8];
    __shared__ int32_t s_lj[kCvList];
    __shared__ double s_ls[kCvList];
    __shared__ int s_ln;
    __shared__ int s_abort;
    __shared__ uint64_t s_ep0;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    int64_t r;
    int h;
    if constexpr (KH == 1) {
        r = blockIdx.x;
        h = 0;
    } else {
        // the two halves of a replicate are 8 workgroups apart (same XCD)
        const int b = (int)blockIdx.x;
        r = (int64_t)(b / 16) * 8 + (b % 8);
        h = (b % 16) / 8;
        if (r >= a.reps) return;
    }
    const int64_t off = r * a.stride;
    double *eta = a.eta + off;
    double *e = a.e + off;
    const double *gr = f.g + off;
    const uint8_t *d8 = a.d8 + off;
    const int32_t *d32 = a.d32 + off;
    const int nch = (int)min(a.stride / CHUNK, (a.n + CHUNK - 1) / CHUNK);
    const int chm = (nch * kCvSplitNum + kCvSplitDen / 2) / kCvSplitDen;
    const int ch_lo = (KH == 2 && h == 1) ? chm : 0;
    const int ch_hi = (KH == 2 && h == 0) ? chm : nch;
    const bool lead = h == 0;                  // owns beta, delta, g12_out
    const bool sums_next = KH == 2 && h == 0;  // e x_{j+1} sums for half 1
    const int64_t tpos = (int64_t)tid * IPT;
    const int64_t T = a.j_end - a.j_begin;
    if (tid == 0) {
        s_ln = 0;
        s_abort = 0;
        s_ep0 = KH == 2 ? ld_relaxed_u64(cv_epoch(a, r)) : 0;
    }
    __syncthreads();
    const uint64_t ep0 = s_ep0;

    // totals of the first coordinate (every half over all chunks, in the
    // same order: the same numbers), and half 1's first carries
    double tw = 0.0, twx = 0.0;
    double k[4] = {0.0, 0.0, 0.0, 0.0};
    if (T > 0) {
        double t4[4];
        fg_sums<BLOCK, IPT>(a, e, gr, a.j_begin, 0, nch, tpos, s_red, s_step, t4);
        tw = t4[2];
        twx = t4[3];
        if (KH == 2 && h == 1) fg_sums<BLOCK, IPT>(a, e, gr, a.j_begin, 0, chm, tpos, s_red, s_step, k);
    }

    double s_prev = 0.0, es_prev = 1.0;
    int64_t jp = -1;
    // the next chunk's e, counts and column bits are loaded during the
    // current one's arithmetic (x1: column j + 1, for the next totals); G
    // is loaded with the chunk itself (fewer registers)
    CvChunk<IPT> cur;
    if (T > 0 && ch_lo < ch_hi)
        cv_load<IPT>(a, e, d8, (int64_t)ch_lo * CHUNK + tpos, a.j_begin, -1,
                     a.j_begin + 1 < a.j_end ? a.j_begin + 1 : -1, cur);
    int par = 0;
    for (int64_t j = a.j_begin; j < a.j_end && !s_abort; ++j) {
        double cj = 0.0, bj = 0.0, dj = 0.0;
        if (lead && tid == 0) {
            cj = a.c[r * a.p + j];
            bj = a.beta[r * a.p + j];
            dj = a.delta[r * a.p + j];
        }
        // carry[2], carry[3] end the pass as sum e w and sum e w x_j up to
        // the end of this half (half 1: over the replicate)
        double acc1 = 0.0, acc2 = 0.0, sa1 = 0.0, sd1 = 0.0, a1 = 0.0, d1 = 0.0;
        double carry[4] = {k[0], k[1], k[2], k[3]};
        for (int ch = ch_lo; ch < ch_hi; ++ch) {
            const int64_t pos = (int64_t)ch * CHUNK + tpos;
            if (cur.px != 0u && s_prev != 0.0) {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if ((cur.px >> i) & 1u) cur.v[i] *= es_prev;
                double2 *dst = reinterpret_cast<double2 *>(e + pos);
#pragma unroll
                for (int i = 0; i < IPT / 2; ++i)
                    dst[i] = make_double2(cur.v[2 * i], cur.v[2 * i + 1]);
            }
            uint32_t dv[IPT];
#pragma unroll
            for (int i = 0; i < IPT; ++i) dv[i] = (cur.d[i / 4] >> (8 * (i % 4))) & 0xffu;
#pragma unroll
            for (int i = 0; i < IPT; ++i)
                if (dv[i] == 255u) dv[i] = (uint32_t)d32[pos + i];
            // G of the training subset at the chunk's positions and w
            double gv[IPT], wv[IPT];
            fg_load_g<IPT>(gr, pos, gv);
            fg_weights<IPT>(cv_bits<IPT>(a, a.p, pos), gv, wv);
            CvChunk<IPT> nx;
            const bool last = ch + 1 == ch_hi;
            const int64_t jn = last ? (j + 1 < a.j_end ? j + 1 : j) : j;
            const int64_t jn1 = jn + 1 < a.j_end ? jn + 1 : -1;
            cv_load<IPT>(a, e, d8, last ? (int64_t)ch_lo * CHUNK + tpos : pos + CHUNK, jn,
                         last ? j : jp, jn1, nx);

            double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const bool xi = (cur.x >> i) & 1u;
                const double ew = cur.v[i] * wv[i];
                t[0] += cur.v[i];
                t[1] += xi ? cur.v[i] : 0.0;
                t[2] += ew;
                t[3] += xi ? ew : 0.0;
                const bool x1 = (cur.x1 >> i) & 1u;
                sa1 += x1 ? ew : 0.0;
                sd1 += (x1 && xi) ? ew : 0.0;
                if (sums_next) {
                    a1 += x1 ? cur.v[i] : 0.0;
                    d1 += (x1 && xi) ? cur.v[i] : 0.0;
                }
            }
            double inc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                inc[c] = dpp_incl_scan(t[c]);
                if (lane == kWave - 1) s_tot[par][w][c] = inc[c];
            }
            __syncthreads();
            double S[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double b, tt;
                wave_totals_prefix<NW>(lane < NW ? s_tot[par][lane][c] : 0.0, w, b, tt);
                S[c] = carry[c] + b + (inc[c] - t[c]);
                carry[c] += tt;
            }
            par ^= 1;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const bool xi = (cur.x >> i) & 1u;
                const double ew = cur.v[i] * wv[i];
                S[0] += cur.v[i];
                S[1] += xi ? cur.v[i] : 0.0;
                S[2] += ew;
                S[3] += xi ? ew : 0.0;
                const uint32_t d = dv[i];
                if (d != 0u) {
                    // G of the training subset at the run end
                    const double gk = gv[i];
                    const double S0 = S[0] + gk * (tw - S[2]);
                    const double S1 = S[1] + gk * (twx - S[3]);
                    const double g = S1 / S0;
                    const double dd = (double)d;
                    acc1 = fma(dd, g, acc1);
                    acc2 = fma(dd, g - g * g, acc2);
                }
            }
            cur = nx;
        }
        double red[6] = {acc1, acc2, sa1, sd1, a1, d1};
        if (sums_next) block_sum<6, BLOCK>(red, s_red);
        else block_sum<4, BLOCK>(*reinterpret_cast<double(*)[4]>(red), s_red);
        if (tid == 0) {
            double g1, g2, step = 0.0;
            bool ok = true;
            double A1 = red[2], D1 = red[3];  // sum e w x_{j+1}, e w x_j x_{j+1}
            double Aw = carry[2], Dw = carry[3];  // sum e w, e w x_j (replicate)
            if constexpr (KH == 2) {
                const int64_t t = j - a.j_begin + 1;
                const uint64_t tag = ((ep0 + (uint64_t)t) << 1) | 1u;
                const int q = (int)(t & 1);
                double h0[15], h1[6];
                if (h == 0) {
                    h0[0] = red[0]; h0[1] = red[1];
                    h0[2] = carry[0]; h0[3] = carry[1]; h0[4] = carry[2]; h0[5] = carry[3];
                    h0[6] = red[4]; h0[7] = red[5]; h0[8] = red[2]; h0[9] = red[3];
                    h0[10] = cj; h0[11] = bj; h0[12] = dj; h0[13] = 0.0; h0[14] = 0.0;
                    u32x4 *sl = cv_slot(a, r, 0, q);
#pragma unroll
                    for (int m = 0; m < 15; ++m) st_pair(sl + m, h0[m], tag);
                    u32x4 rr[6];
                    ok = wait_pairs<6>(cv_slot(a, r, 1, q), tag, a.hdr, rr);
#pragma unroll
                    for (int m = 0; m < 6; ++m) h1[m] = pair_value(rr[m]);
                } else {
                    h1[0] = red[0]; h1[1] = red[1]; h1[2] = carry[2]; h1[3] = carry[3];
                    h1[4] = red[2]; h1[5] = red[3];
                    u32x4 *sl = cv_slot(a, r, 1, q);
#pragma unroll
                    for (int m = 0; m < 6; ++m) st_pair(sl + m, h1[m], tag);
                    u32x4 rr[15];
                    ok = wait_pairs<15>(cv_slot(a, r, 0, q), tag, a.hdr, rr);
#pragma unroll
                    for (int m = 0; m < 15; ++m) h0[m] = pair_value(rr[m]);
                    cj = h0[10]; bj = h0[11]; dj = h0[12];
                }
                g1 = cj - (h0[0] + h1[0]);
                g2 = -(h0[1] + h1[1]);
                // the replicate's sums, the same numbers in both halves
                Aw = h1[2];
                Dw = h1[3];
                A1 = h0[8] + h1[4];
                D1 = h0[9] + h1[5];
                if (ok) ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &step);
                if (h == 1) {
                    const double em = expm1(step);
                    s_step[4] = fma(em, h0[3], h0[2]);
                    s_step[5] = fma(em, h0[7], h0[6]);
                    s_step[6] = fma(em, h0[5], h0[4]);
                    s_step[7] = fma(em, h0[9], h0[8]);
                }
            } else {
                g1 = cj - red[0];
                g2 = -red[1];
                ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &step);
            }
            if (!ok) s_abort = 1;
            if (lead && ok) {
                a.beta[r * a.p + j] = bj;
                a.delta[r * a.p + j] = dj;
                if (a.g12_out) {
                    double *o = a.g12_out + (r * a.p + j) * 3;
                    o[0] = g1;
                    o[1] = g2;
                    o[2] = step;
                }
            }
            const double em = expm1(step);
            s_step[0] = step;
            s_step[1] = exp(step);
            s_step[2] = fma(em, Dw, Aw);
            s_step[3] = fma(em, D1, A1);
            if (step != 0.0) {
                s_lj[s_ln] = (int32_t)j;
                s_ls[s_ln] = step;
                s_ln = s_ln + 1;
            }
        }
        __syncthreads();
        s_prev = s_step[0];
        es_prev = s_step[1];
        tw = s_step[2];
        twx = s_step[3];
        if (KH == 2 && h == 1) {
#pragma unroll
            for (int c = 0; c < 4; ++c) k[c] = s_step[4 + c];
        }
        jp = j;
        if (s_ln == kCvList) {
            cv_apply_steps<IPT, BLOCK>(a, eta, e, a.train_s + off, s_lj, s_ls, kCvList, ch_lo,
                                       ch_hi, tpos, false);
            __syncthreads();
            if (tid == 0) s_ln = 0;
            __syncthreads();
        }
    }
    cv_apply_steps<IPT, BLOCK>(a, eta, e, a.train_s + off, s_lj, s_ls, s_ln, ch_lo, ch_hi, tpos,
                               true);
    // half 0 has seen half 1's last publication, made after half 1 read the
    // epoch: the next launch's tags start after this launch's
    if (KH == 2 && h == 0 && tid == 0 && T > 0 && !s_abort)
        st_relaxed_u64(cv_epoch(a, r), ep0 + (uint64_t)T + 1);
}

// Fine-Gray training and held-out log pseudo-likelihoods (eq. fg_l on each
// subset): a first pass sums the weighted totals of both subsets, the
// second scans e and e w of each subset and takes d log S0 at the run ends
// of each subset's events (S0 = prefix + G (total - weighted prefix)).
__global__ __launch_bounds__(kCvBlock) void k_cv_loglik_fg(int64_t n, int64_t stride,
                                                           const int32_t *perm,
                                                           const int8_t *status,
                                                           const double *eta, const double *e,
                                                           const uint8_t *train_s,
                                                           const uint8_t *d8, const int32_t *d32,
                                                           const uint8_t *d8_r,
                                                           const int32_t *d32_r,
                                                           const double *w_r, const double *g_r,
                                                           const double *g_h, double *out)
{
    __shared__ double s_tot[kCvWaves][4];
    __shared__ double s_red[kCvWaves * 4];
    __shared__ double s_t[2];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t r = blockIdx.x;
    const int64_t off = r * stride;
    // pass 1: sum e w over the training subset and over the held-out one
    double tt[2] = {0.0, 0.0};
    for (int64_t k = tid; k < n; k += kCvBlock) {
        const bool tr = train_s[off + k] != 0;
        if (tr) {
            tt[0] += e[off + k] * w_r[off + k];
        } else if (status[perm[k]] == 2) {
            tt[1] += exp(eta[off + k]) / g_h[off + k];
        }
    }
    block_sum<2, kCvBlock>(tt, s_red);
    if (tid == 0) {
        s_t[0] = tt[0];
        s_t[1] = tt[1];
    }
    __syncthreads();
    const double T0 = s_t[0], T1 = s_t[1];
    double carry[4] = {0.0, 0.0, 0.0, 0.0}, lt = 0.0, lh = 0.0;
    for (int64_t base = 0; base < n; base += kCvBlock) {
        const int64_t k = base + tid;
        double v[4] = {0.0, 0.0, 0.0, 0.0};  // e_t, e_t w_t, e_h, e_h w_h
        double x = 0.0;
        int dt = 0, dall = 0;
        bool tr = false, ev = false;
        if (k < n) {
            tr = train_s[off + k] != 0;
            x = eta[off + k];
            const int8_t st = status[perm[k]];
            ev = st == 1;
            if (tr) {
                v[0] = e[off + k];
                v[1] = v[0] * w_r[off + k];
            } else {
                v[2] = exp(x);
                v[3] = st == 2 ? v[2] / g_h[off + k] : 0.0;
            }
            dt = d8_r[off + k];
            if (dt == 255) dt = d32_r[off + k];
            dall = d8[k];
            if (dall == 255) dall = d32[k];
        }
        double inc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            inc[c] = dpp_incl_scan(v[c]);
            if (lane == kWave - 1) s_tot[w][c] = inc[c];
        }
        __syncthreads();
        double S[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double b, t;
            wave_totals_prefix(lane < kCvWaves ? s_tot[lane][c] : 0.0, w, b, t);
            S[c] = carry[c] + b + inc[c];
            carry[c] += t;
        }
        const int dh = dall - dt;
        if (ev) {
            if (tr) lt += x;
            else lh += x;
        }
        if (dt > 0) lt -= (double)dt * log(S[0] + g_r[off + k] * (T0 - S[1]));
        if (dh > 0) lh -= (double)dh * log(S[2] + g_h[off + k] * (T1 - S[3]));
        __syncthreads();
    }
    double red[2] = {lt, lh};
    block_sum<2, kCvBlock>(red, s_red);
    if (tid == 0) {
        out[2 * r] = red[0];
        out[2 * r + 1] = red[1];
    }
}

// ---------------------------------------------------------------- likelihood
// Per replicate: the training log-likelihood (the e of the replicate, its
// event counts) and the held-out one (exp(eta) of the held-out subjects,
// the full data set's counts minus the training ones), each
// sum over events of eta minus sum over run ends of d log S0.
__global__ __launch_bounds__(kCvBlock) void k_cv_loglik(int32_t model, int64_t n,
                                                        int64_t stride, const int32_t *perm,
                                                        const int8_t *status,
                                                        const double *eta, const double *e,
                                                        const uint8_t *train_s,
                                                        const uint8_t *d8, const int32_t *d32,
                                                        const uint8_t *d8_r,
                                                        const int32_t *d32_r, double *out)
{
    __shared__ double s_tot[kCvWaves][2];
    __shared__ double s_red[kCvWaves * 2];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    const int64_t r = blockIdx.x;
    const int64_t off = r * stride;
    double carry0 = 0.0, carry1 = 0.0, lt = 0.0, lh = 0.0;
    for (int64_t base = 0; base < n; base += kCvBlock) {
        const int64_t k = base + tid;
        double et = 0.0, eh = 0.0, x = 0.0;
        int dt = 0, dall = 0;
        bool tr = false, ev = false;
        if (k < n) {
            tr = train_s[off + k] != 0;
            x = eta[off + k];
            et = e[off + k];
            eh = tr ? 0.0 : exp(x);
            ev = cv_event(model, status[perm[k]]);
            dt = d8_r[off + k];
            if (dt == 255) dt = d32_r[off + k];
            dall = d8[k];
            if (dall == 255) dall = d32[k];
        }
        const double i0 = dpp_incl_scan(et);
        const double i1 = dpp_incl_scan(eh);
        if (lane == kWave - 1) {
            s_tot[w][0] = i0;
            s_tot[w][1] = i1;
        }
        __syncthreads();
        double b0, b1, T0, T1;
        wave_totals_prefix(lane < kCvWaves ? s_tot[lane][0] : 0.0, w, b0, T0);
        wave_totals_prefix(lane < kCvWaves ? s_tot[lane][1] : 0.0, w, b1, T1);
        const double p0 = carry0 + b0, p1 = carry1 + b1;
        const double c0 = carry0 + T0, c1 = carry1 + T1;
        const double S0t = p0 + i0, S0h = p1 + i1;
        const int dh = dall - dt;
        if (ev) {
            if (tr) lt += x;
            else lh += x;
        }
        if (dt > 0) lt -= (double)dt * log(S0t);
        if (dh > 0) lh -= (double)dh * log(S0h);
        carry0 = c0;
        carry1 = c1;
        __syncthreads();
    }
    double red[2] = {lt, lh};
    block_sum<2, kCvBlock>(red, s_red);
    if (tid == 0) {
        out[2 * r] = red[0];
        out[2 * r + 1] = red[1];
    }
}

int grid_of(int64_t n, int64_t cap) { return (int)std::max<int64_t>(1, std::min(cap, ceil_div(n, 256))); }

// The choice of the penalty strength (Sec. 2.8): thread g sums the held-out
// scores of strength g over the replicates in replicate order; thread 0 then
// takes the first strength with the largest mean (NaN means never win).
__global__ __launch_bounds__(256) void k_cv_select(int32_t n_gamma, int32_t reps,
                                                   const double *scores, double *mean,
                                                   int32_t *best)
{
    for (int32_t g0 = 0; g0 < n_gamma; g0 += 256) {
        const int32_t g = g0 + (int32_t)threadIdx.x;
        if (g < n_gamma) {
            const double *row = scores + (int64_t)g * 2 * reps;
            double s = 0.0;
            for (int32_t r = 0; r < reps; ++r) s += row[2 * r + 1];
            mean[g] = s / (double)reps;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t b = -1;
        double bv = 0.0;
        for (int32_t g = 0; g < n_gamma; ++g) {
            const double v = mean[g];
            if (v == v && (b < 0 || v > bv)) {
                b = g;
                bv = v;
            }
        }
        *best = b;
    }
}

}  // namespace

int32_t launch_cv_select(int32_t n_gamma, int32_t reps, const double *scores, double *mean,
                         int32_t *best, hipStream_t s)
{
    hipLaunchKernelGGL(k_cv_select, dim3(1), dim3(256), 0, s, n_gamma, reps, scores, mean,
                       best);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int64_t cv_stride(int64_t n) { return ceil_div(n, kCvAlign) * kCvAlign; }

int32_t launch_cv_prepare(int32_t model, int64_t n, int64_t p, int32_t reps, const int32_t *perm,
                          const int8_t *status, const double *y, const uint8_t *d8,
                          const uint8_t *train, const int64_t *col_ptr,
                          const int32_t *rows_sorted, uint8_t *train_s, uint8_t *d8_r,
                          int32_t *d32_r, uint32_t *xbits, double *c_r, double *w_r,
                          double *g_r, double *g_h, void *ws, hipStream_t s)
{
    const int64_t stride = cv_stride(n);
    const int64_t words = stride / 32;
    uint32_t *evbits = reinterpret_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(k_cv_prep, dim3(reps), dim3(kCvBlock), 0, s, model, n, stride, perm,
                       status, train, d8, train_s, d8_r, d32_r, evbits);
    SS_LAUNCH_CHECK();
    const int64_t cols = model == SS_FINE_GRAY ? p + 1 : p;
    hipLaunchKernelGGL(k_cv_fill, dim3(grid_of(cols * words, 8192)), dim3(256), 0, s, xbits,
                       cols * words);
    SS_LAUNCH_CHECK();
    if (model == SS_FINE_GRAY) {
        hipLaunchKernelGGL(k_cv_comp_bits, dim3(grid_of(n, 256)), dim3(256), 0, s, n, perm,
                           status, xbits + p * words);
        SS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cv_bits, dim3((unsigned)std::min<int64_t>(p, 65535)), dim3(256), 0, s,
                       p, words, col_ptr, rows_sorted, xbits);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cv_c, dim3((unsigned)p, (unsigned)reps), dim3(256), 0, s, p, words,
                       xbits, evbits, c_r);
    SS_LAUNCH_CHECK();
    if (model == SS_FINE_GRAY) {
        hipLaunchKernelGGL(k_cv_km, dim3(reps), dim3(kCvBlock), 0, s, n, stride, perm, status, y,
                           train_s, w_r, g_r, g_h);
        SS_LAUNCH_CHECK();
    }
    return SS_OK;
}

int32_t launch_cv_exp(int64_t n, int32_t reps, const double *eta, const uint8_t *train_s,
                      double *e, hipStream_t s)
{
    const int64_t total = cv_stride(n) * reps;
    hipLaunchKernelGGL(k_cv_exp, dim3(grid_of(total, 8192)), dim3(256), 0, s, total, eta,
                       train_s, e);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

size_t cv_ws_bytes(int32_t reps) { return 256 + (size_t)reps * kCvXchBytes; }

int32_t launch_cv_sweep(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                        int32_t reps, int64_t j_begin, int64_t j_end, double *eta, double *e,
                        const uint8_t *d8_r, const int32_t *d32_r, const uint8_t *train_s,
                        const uint32_t *xbits, const double *c_r, const double *w_r,
                        const double *g_r, double *beta, double *delta, double *g12_out,
                        void *ws, hipStream_t s)
{
    CvArgs a;
    a.n = n;
    a.p = p;
    a.stride = cv_stride(n);
    a.j_begin = j_begin;
    a.j_end = j_end;
    a.reps = reps;
    a.penalty = penalty;
    a.lambda = lambda;
    a.eta = eta;
    a.e = e;
    a.d8 = d8_r;
    a.d32 = d32_r;
    a.train_s = train_s;
    a.xbits = reinterpret_cast<const uint8_t *>(xbits);
    a.c = c_r;
    a.beta = beta;
    a.delta = delta;
    a.g12_out = g12_out;
    a.hdr = reinterpret_cast<WsHeader *>(ws);
    a.xch = reinterpret_cast<char *>(ws) + 256;
    // two workgroups per replicate when all of them fit on the device at
    // once (a cooperative launch checks it); one per replicate otherwise.
    // SURVSCAN_CV_HALVES=1 forces one.
    const char *env = getenv("SURVSCAN_CV_HALVES");
    const bool allow2 = !(env && env[0] == '1');
    (void)w_r;  // the sweep derives w from G (the same division)
    if (model == SS_FINE_GRAY) {
        CvFgArgs f;
        f.a = a;
        f.g = g_r;
        if (allow2) {
            int dev = 0, cus = 0, coop = 0, per_cu = 0;
            SS_HIP_CHECK(hipGetDevice(&dev));
            SS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            SS_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
            void *k = reinterpret_cast<void *>(k_cv_sweep_fg<kCvFgBlock, kCvFgIpt, 2>);
            SS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kCvFgBlock, 0));
            const int64_t G = 16 * ceil_div(reps, 8);
            if (coop && G <= (int64_t)per_cu * cus) {
                void *args[] = {&f};
                SS_HIP_CHECK(hipLaunchCooperativeKernel(k, dim3((unsigned)G), dim3(kCvFgBlock),
                                                        args, 0, s));
                return SS_OK;
            }
        }
        hipLaunchKernelGGL((k_cv_sweep_fg<kCvFgBlock, kCvFgIpt, 1>), dim3(reps), dim3(kCvFgBlock),
                           0, s, f);
        SS_LAUNCH_CHECK();
        return SS_OK;
    }
    if (allow2) {
        int dev = 0, cus = 0, coop = 0, per_cu = 0;
        SS_HIP_CHECK(hipGetDevice(&dev));
        SS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        SS_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        void *k = reinterpret_cast<void *>(k_cv_sweep<kCvCoxBlock, 8, 2>);
        SS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kCvCoxBlock, 0));
        const int64_t G = 16 * ceil_div(reps, 8);
        if (coop && G <= (int64_t)per_cu * cus) {
            void *args[] = {&a};
            SS_HIP_CHECK(hipLaunchCooperativeKernel(k, dim3((unsigned)G), dim3(kCvCoxBlock), args,
                                                    0, s));
            return SS_OK;
        }
    }
    hipLaunchKernelGGL((k_cv_sweep<kCvCoxBlock, 8, 1>), dim3(reps), dim3(kCvCoxBlock), 0, s, a);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_cv_loglik(int32_t model, int64_t n, int32_t reps, const int32_t *perm,
                         const int8_t *status, const double *eta, const double *e,
                         const uint8_t *train_s, const uint8_t *d8, const int32_t *d32,
                         const uint8_t *d8_r, const int32_t *d32_r, const double *w_r,
                         const double *g_r, const double *g_h, double *out, hipStream_t s)
{
    if (model == SS_FINE_GRAY) {
        hipLaunchKernelGGL(k_cv_loglik_fg, dim3(reps), dim3(kCvBlock), 0, s, n, cv_stride(n),
                           perm, status, eta, e, train_s, d8, d32, d8_r, d32_r, w_r, g_r, g_h,
                           out);
        SS_LAUNCH_CHECK();
        return SS_OK;
    }
    hipLaunchKernelGGL(k_cv_loglik, dim3(reps), dim3(kCvBlock), 0, s, model, n, cv_stride(n),
                       perm, status, eta, e, train_s, d8, d32, d8_r, d32_r, out);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace ss
