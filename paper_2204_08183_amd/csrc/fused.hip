// Fused coordinate kernels for gfx950: the sparse update of X beta (step
// (1) of Sec. 2.7), the single-pass tuple scan with decoupled look-back,
// the element-wise transform with the event counts and the reduction
// (steps (2)-(4), fused as in Fig. 3), and the coordinate update in the
// last tile (Fig. 4's conditional kernel, Secs. 2.3-2.4).
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
#include "ss_internal.h"

namespace ss {

namespace {

template <int NC>
struct Vec {
    double v[NC];
};

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

// Decoupled look-back (single-pass chained scan, Sec. 2.6): wave 0 of tile
// `tile` walks back over its predecessors 64 at a time until it meets an
// inclusive prefix.  Returns the tile's exclusive prefix in every lane of
// wave 0.  Every predecessor took its ticket earlier and publishes its
// aggregate without waiting, so the wait ends; it is still bounded.
template <int NC>
__device__ void look_back(const TileState *tiles, int64_t tile, uint64_t epoch,
                          WsHeader *hdr, double (&excl)[NC])
{
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < NC; ++c) excl[c] = 0.0;
    int64_t top = tile - 1;
    uint32_t spins = 0;
    bool give_up = false;
    while (top >= 0) {
        const int64_t t = top - lane;
        uint64_t state = kStateInc;  // before tile 0: empty inclusive prefix
        // every lane runs the same iterations, so the loop stays wave-uniform
        for (;;) {
            if (t >= 0) {
                const uint64_t f = ld_flag(&tiles[t].flag);
                state = (f >> 2) == epoch ? (f & 3u) : 0u;
            }
            if (!__any(state == 0)) break;
            if (++spins > kSpinLimit) { give_up = true; break; }
            __builtin_amdgcn_s_sleep(1);
        }
        if (give_up) {
            if (lane == 0) __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        order_acquire();  // payload loads stay after the flag loads
        const uint64_t inc_mask = __ballot(state == kStateInc);
        const int first_inc = inc_mask ? __ffsll((unsigned long long)inc_mask) - 1 : kWave;
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = 0.0;
        if (t >= 0 && lane <= first_inc) {
            const double *src = (state == kStateInc) ? tiles[t].inc : tiles[t].agg;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = ld_relaxed(src + c);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) excl[c] += wave_sum(v[c]);
        if (inc_mask) break;
        top -= kWave;
    }
}

template <int NC>
__device__ __forceinline__ void publish(TileState *ts, const double (&val)[NC],
                                        bool inclusive, uint64_t epoch)
{
    double *dst = inclusive ? ts->inc : ts->agg;
#pragma unroll
    for (int c = 0; c < NC; ++c) st_relaxed(dst + c, val[c]);
    order_release();  // the payload is at the coherence point before the flag
    st_flag(&ts->flag, (epoch << 2) | (inclusive ? kStateInc : kStateAgg));
}

// Applies a pending step of column jprev to eta and e inside [t0, t1).
template <int BLOCK, bool VALS>
__device__ __forceinline__ void apply_prev(const FusedCall &a, int64_t chunk0,
                                           int64_t chunk1)
{
    const double st = *a.step_prev;
    if (st == 0.0) return;
    const int64_t cb = a.col.col_ptr[a.jprev];
    const int32_t *cp = a.col.chunk_ptr + (int64_t)a.jprev * a.col.nchunk1;
    const int32_t lo = cp[chunk0];
    const int32_t hi = cp[chunk1];
    for (int32_t o = lo + (int32_t)threadIdx.x; o < hi; o += BLOCK) {
        const int32_t r = a.col.rows[cb + o];
        const double x = VALS ? a.col.vals[cb + o] : 1.0;
        const double et = a.eta[r] + x * st;
        a.eta[r] = et;
        a.e[r] = exp(et);
    }
}

// Scatters the non-zeros of column j inside the tile into s_x (zeroed).
template <int BLOCK, int TILE, bool VALS>
__device__ __forceinline__ void load_column(const FusedCall &a, int64_t t0,
                                            int64_t chunk0, int64_t chunk1,
                                            double *s_x)
{
    for (int i = threadIdx.x; i < TILE; i += BLOCK) s_x[i] = 0.0;
    __syncthreads();
    if (a.j >= 0) {
        const int64_t cb = a.col.col_ptr[a.j];
        const int32_t *cp = a.col.chunk_ptr + (int64_t)a.j * a.col.nchunk1;
        const int32_t lo = cp[chunk0];
        const int32_t hi = cp[chunk1];
        for (int32_t o = lo + (int32_t)threadIdx.x; o < hi; o += BLOCK) {
            const int32_t r = a.col.rows[cb + o];
            s_x[r - t0] = VALS ? a.col.vals[cb + o] : 1.0;
        }
    }
    __syncthreads();
}

// Last tile: fixed-order sum of the per-tile partials, then g', g'', the
// likelihood or the coordinate update, then reset of the launch counters.
template <int BLOCK>
__device__ void finish(const FusedCall &a, const WsView &ws, int64_t ntiles,
                       double *s_red)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = threadIdx.x; t < ntiles; t += BLOCK) {
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += ld_relaxed(ws.partials + 4 * t + c);
    }
    double btc = 0.0;
    if (a.beta_ll) {
        for (int64_t q = threadIdx.x; q < a.p; q += BLOCK) btc += a.beta_ll[q] * a.c[q];
    }
    double all[4] = {acc[0], acc[1], acc[2], btc};
    block_sum<4, BLOCK>(all, s_red);
    if (threadIdx.x == 0) {
        const double A = all[0], B = all[1], L = all[2];
        if (a.beta_ll) {
            a.out[0] = all[3] - L;
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
        }
        WsHeader *h = ws.hdr;
        st_relaxed_u32(&h->ticket, 0u);
        st_relaxed_u32(&h->done, 0u);
        const uint64_t ep = ld_relaxed_u64(&h->epoch);
        st_relaxed_u64(&h->epoch, ep + 1);
    }
}

// The fused scan -> transform -> reduce kernel (one coordinate).
// MODEL: SS_COX (3 tuple components) or SS_FINE_GRAY (6).
template <int BLOCK, int IPT, int MODEL, bool VALS, bool PREV>
__global__ __launch_bounds__(BLOCK) void k_fused(FusedCall a, WsView ws,
                                                 int64_t ntiles)
{
    constexpr int TILE = BLOCK * IPT;
    constexpr int NC = MODEL == SS_FINE_GRAY ? 6 : 3;
    constexpr int NW = BLOCK / kWave;
    static_assert(TILE % SS_CHUNK == 0, "tile must be whole chunks");

    __shared__ double s_x[TILE];
    __shared__ double s_wsum[NW][NC];
    __shared__ double s_excl[NC];
    __shared__ double s_red[NW * 4];
    __shared__ int64_t s_tile;
    __shared__ uint64_t s_epoch;
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;

    if (tid == 0) {
        s_tile = (int64_t)fetch_add_relaxed(&ws.hdr->ticket, 1u);
        s_epoch = ld_relaxed_u64(&ws.hdr->epoch);
    }
    __syncthreads();
    const int64_t tile = s_tile;
    const uint64_t epoch = s_epoch;
    const int64_t t0 = tile * TILE;
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = t0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + TILE / SS_CHUNK, nchunk);

    if (PREV) {
        apply_prev<BLOCK, VALS>(a, chunk0, chunk1);
        __syncthreads();
    }
    load_column<BLOCK, TILE, VALS>(a, t0, chunk0, chunk1, s_x);

    // ---- load the tile (vector loads when the tile is full)
    const int64_t base = t0 + (int64_t)tid * IPT;
    const bool full = t0 + TILE <= a.n;
    double ev[IPT];
    double xv[IPT];
    double wv[MODEL == SS_FINE_GRAY ? IPT : 1];
    int dk[IPT];
    if (full) {
        const double2 *ep = reinterpret_cast<const double2 *>(a.e + base);
#pragma unroll
        for (int q = 0; q < IPT / 2; ++q) {
            const double2 v = ep[q];
            ev[2 * q] = v.x;
            ev[2 * q + 1] = v.y;
        }
        if (IPT >= 8) {
            const uint64_t *dp = reinterpret_cast<const uint64_t *>(a.d8 + base);
#pragma unroll
            for (int q = 0; q < IPT / 8; ++q) {
                const uint64_t dd = dp[q];
#pragma unroll
                for (int b = 0; b < 8; ++b) dk[8 * q + b] = (int)((dd >> (8 * b)) & 255u);
            }
        } else {
            const uint32_t dd = *reinterpret_cast<const uint32_t *>(a.d8 + base);
#pragma unroll
            for (int b = 0; b < IPT; ++b) dk[b] = (int)((dd >> (8 * b)) & 255u);
        }
        if (MODEL == SS_FINE_GRAY) {
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
            const int64_t k = base + i;
            const bool ok = k < a.n;
            ev[i] = ok ? a.e[k] : 0.0;
            dk[i] = ok ? (int)a.d8[k] : 0;
            if (MODEL == SS_FINE_GRAY) wv[i] = ok ? a.w_comp[k] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) xv[i] = s_x[tid * IPT + i];

    // ---- thread totals of the tuple
    double run[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) run[c] = 0.0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const double ex = ev[i] * xv[i];
        run[0] += ev[i];
        run[1] += ex;
        run[2] += ex * xv[i];
        if (MODEL == SS_FINE_GRAY) {
            const double ew = ev[i] * wv[i];
            const double exw = ew * xv[i];
            run[3] += ew;
            run[4] += exw;
            run[5] += exw * xv[i];
        }
    }

    // ---- block scan of the thread totals
    double incl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) incl[c] = run[c];
    wave_inclusive_scan<NC>(incl);
    if (lane == kWave - 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) s_wsum[w][c] = incl[c];
    }
    __syncthreads();
    double texcl[NC];  // exclusive prefix of this thread inside the tile
    double agg[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double before = 0.0, total = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q < w) before += s_wsum[q][c];
            total += s_wsum[q][c];
        }
        texcl[c] = before + incl[c] - run[c];
        agg[c] = total;
    }

    // ---- decoupled look-back for the tile's exclusive prefix
    if (w == 0) {
        TileState *ts = ws.tiles + tile;
        if (tile == 0) {
            if (lane == 0) publish<NC>(ts, agg, true, epoch);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < NC; ++c) s_excl[c] = 0.0;
            }
        } else {
            if (lane == 0) publish<NC>(ts, agg, false, epoch);
            double ex[NC];
            look_back<NC>(ws.tiles, tile, epoch, ws.hdr, ex);
            if (lane == 0) {
                double inc[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) inc[c] = ex[c] + agg[c];
                publish<NC>(ts, inc, true, epoch);
#pragma unroll
                for (int c = 0; c < NC; ++c) s_excl[c] = ex[c];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) texcl[c] += s_excl[c];

    double tot[3] = {0.0, 0.0, 0.0};
    if (MODEL == SS_FINE_GRAY) {
#pragma unroll
        for (int c = 0; c < 3; ++c) tot[c] = ws.hdr->fg_tot[c];
    }

    // ---- running prefix, transform at run ends, reduction
    double acc[3] = {0.0, 0.0, 0.0};
    double S[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) S[c] = texcl[c];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const double ex = ev[i] * xv[i];
        S[0] += ev[i];
        S[1] += ex;
        S[2] += ex * xv[i];
        if (MODEL == SS_FINE_GRAY) {
            const double ew = ev[i] * wv[i];
            const double exw = ew * xv[i];
            S[3] += ew;
            S[4] += exw;
            S[5] += exw * xv[i];
        }
        int d = dk[i];
        if (d != 0) {
            const int64_t k = base + i;
            if (d == 255) d = a.d32[k];
            double S0 = S[0], S1 = S[1], S2 = S[2];
            if (MODEL == SS_FINE_GRAY) {
                const double g = a.g_end[k];
                S0 += g * (tot[0] - S[3]);
                S1 += g * (tot[1] - S[4]);
                S2 += g * (tot[2] - S[5]);
            }
            const double r = 1.0 / S0;
            const double G = S1 * r;
            const double H = S2 * r;
            const double dd = (double)d;
            acc[0] += dd * G;
            acc[1] += dd * (H - G * G);
            if (a.want_log) acc[2] += dd * log(S0);
        }
    }
    block_sum<3, BLOCK>(acc, s_red);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) st_relaxed(ws.partials + 4 * tile + c, acc[c]);
        order_release();
        const uint32_t prev = fetch_add_relaxed(&ws.hdr->done, 1u);
        s_last = prev == (uint32_t)(ntiles - 1);
    }
    __syncthreads();
    if (s_last) {
        order_acquire();
        finish<BLOCK>(a, ws, ntiles, s_red);
    }
}

// Fine-Gray totals pass: applies the pending step (a1) and reduces
// sum_r e_r x_r^m w_comp_r (m = 0, 1, 2) into hdr->fg_tot.
template <int BLOCK, int IPT, bool VALS, bool PREV>
__global__ __launch_bounds__(BLOCK) void k_fg_totals(FusedCall a, WsView ws,
                                                     int64_t ntiles)
{
    constexpr int TILE = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ double s_x[TILE];
    __shared__ double s_red[NW * 4];
    __shared__ int s_last;
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * TILE;
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = t0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + TILE / SS_CHUNK, nchunk);
    if (PREV) {
        apply_prev<BLOCK, VALS>(a, chunk0, chunk1);
        __syncthreads();
    }
    load_column<BLOCK, TILE, VALS>(a, t0, chunk0, chunk1, s_x);
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t base = t0 + (int64_t)threadIdx.x * IPT;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t k = base + i;
        if (k < a.n) {
            const double ew = a.e[k] * a.w_comp[k];
            const double xk = s_x[threadIdx.x * IPT + i];
            acc[0] += ew;
            acc[1] += ew * xk;
            acc[2] += ew * xk * xk;
        }
    }
    block_sum<3, BLOCK>(acc, s_red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) st_relaxed(ws.fg_partials + 4 * tile + c, acc[c]);
        order_release();
        const uint32_t prev = fetch_add_relaxed(&ws.hdr->fg_done, 1u);
        s_last = prev == (uint32_t)(ntiles - 1);
    }
    __syncthreads();
    if (s_last) {
        order_acquire();
        double t[3] = {0.0, 0.0, 0.0};
        for (int64_t q = threadIdx.x; q < ntiles; q += BLOCK) {
#pragma unroll
            for (int c = 0; c < 3; ++c) t[c] += ld_relaxed(ws.fg_partials + 4 * q + c);
        }
        block_sum<3, BLOCK>(t, s_red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) ws.hdr->fg_tot[c] = t[c];
            st_relaxed_u32(&ws.hdr->fg_done, 0u);
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

size_t fused_ws_bytes(int64_t n)
{
    const int64_t tiles = ceil_div(n, SS_CHUNK) + 1;
    size_t b = sizeof(WsHeader);
    b = align_up(b + sizeof(TileState) * (size_t)tiles, 256);
    b = align_up(b + sizeof(double) * 4 * (size_t)tiles, 256);
    b = align_up(b + sizeof(double) * 4 * (size_t)tiles, 256);
    return b;
}

bool fused_ws_view(void *ws, size_t ws_bytes, int64_t n, WsView *v)
{
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < fused_ws_bytes(n)) return false;
    const int64_t tiles = ceil_div(n, SS_CHUNK) + 1;
    char *p = (char *)ws;
    v->hdr = (WsHeader *)p;
    size_t off = sizeof(WsHeader);
    v->tiles = (TileState *)(p + off);
    off = align_up(off + sizeof(TileState) * (size_t)tiles, 256);
    v->partials = (double *)(p + off);
    off = align_up(off + sizeof(double) * 4 * (size_t)tiles, 256);
    v->fg_partials = (double *)(p + off);
    v->max_tiles = tiles;
    return true;
}

namespace {

// Items per thread by problem size: small problems take small tiles so that
// every CU gets work, large ones take big tiles to amortise the per-tile
// look-back and bookkeeping.
int pick_ipt(int64_t n)
{
    if (n <= (int64_t)4 << 20) return 4;
    if (n <= (int64_t)32 << 20) return 8;
    return 16;
}

template <int IPT, int MODEL, bool VALS, bool PREV>
void launch_fused_t(const FusedCall &a, const WsView &ws, int64_t ntiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_fused<kBlock, IPT, MODEL, VALS, PREV>), dim3((unsigned)ntiles),
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

template <int IPT>
int32_t launch_fused_ipt(const FusedCall &a, const WsView &ws, hipStream_t s)
{
    const int64_t ntiles = ceil_div(a.n, (int64_t)kBlock * IPT);
    if (ntiles > ws.max_tiles) return SS_EWORKSPACE;
    const bool vals = a.col.vals != nullptr;
    const bool prev = a.jprev >= 0;
    FusedCall b = a;
    if (a.model == SS_FINE_GRAY) {
        // totals pass (and the pending a1 update), then the scan pass
        launch_fg_totals_t<IPT>(a, ws, ntiles, vals, prev, s);
        SS_LAUNCH_CHECK();
        b.jprev = -1;
        if (vals) launch_fused_t<IPT, SS_FINE_GRAY, true, false>(b, ws, ntiles, s);
        else      launch_fused_t<IPT, SS_FINE_GRAY, false, false>(b, ws, ntiles, s);
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

}  // namespace

int32_t launch_fused(const FusedCall &a, const WsView &ws, hipStream_t s)
{
    switch (pick_ipt(a.n)) {
    case 4: return launch_fused_ipt<4>(a, ws, s);
    case 8: return launch_fused_ipt<8>(a, ws, s);
    default: return launch_fused_ipt<16>(a, ws, s);
    }
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
