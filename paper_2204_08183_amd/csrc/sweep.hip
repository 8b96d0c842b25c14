// Persistent cyclic-coordinate-descent sweep for gfx950: the workflow of
// Fig. 4 (sparse update -> fused gradient/Hessian -> conditional update,
// for j = 1..P) in ONE cooperative launch, with no host round trip and no
// per-coordinate launch.
//
// Every workgroup owns a segment of S = BLOCK*IPT consecutive sorted
// positions for the whole sweep; e (and, for Fine-Gray, w and G) of its
// segment stay in registers, and only the rows that an update touches are
// patched.  Per coordinate j the workgroups exchange data twice:
//   1. all-to-all: each publishes the tuple aggregate of its segment, then
//      sums the aggregates of the segments before it (its exclusive prefix
//      of the tuple scan, Sec. 2.7) and, for Fine-Gray, of all segments (the
//      totals that turn the inclusive prefix of e*w into the suffix sum of
//      eq. fg_g) -- a fixed-order sum, so results are deterministic;
//   2. all-to-one-to-all: each publishes its partial sums of
//      d*G, d*(H - G^2), d*log S0; workgroup 0 adds them in order, takes the
//      coordinate update (Secs. 2.3-2.4) and broadcasts the step through one
//      flag per workgroup.
// All exchanged values go through agent-scope atomic loads/stores with
// order-only fences (no L2 flush or invalidate), and every flag carries the
// launch epoch of the coordinate, so nothing is cleared between steps.
// Every wait is bounded; a timed-out wait sets the workspace error word and
// every workgroup leaves at its next wait.
#include "ss_device.h"

namespace ss {

namespace {

using namespace dev;

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

// Waits (one thread) until *f == want.  Returns false if the wait gave up or
// another workgroup already did.
__device__ bool wait_flag(const uint64_t *f, uint64_t want, WsHeader *hdr)
{
    uint32_t spins = 0;
    while (ld_flag(f) != want) {
        if ((++spins & 31u) == 0 && ld_relaxed_u32(&hdr->error)) return false;
        if (spins > kSpinLimit) {
            __hip_atomic_store(&hdr->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
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
    __shared__ double s_wsum[NW][NC];
    __shared__ double s_red[NW * 8];
    __shared__ double s_bc[8];
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

    // ---- the segment's data into registers for the whole sweep
    double ev[IPT];
    int dk[IPT];
    double wv[FG ? IPT : 1];
    double gv[FG ? IPT : 1];
    if (cnt == S) {
        const double2 *ep = reinterpret_cast<const double2 *>(a.e + base);
#pragma unroll
        for (int q = 0; q < IPT / 2; ++q) {
            const double2 v = ep[q];
            ev[2 * q] = v.x;
            ev[2 * q + 1] = v.y;
        }
        uint8_t db[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) db[i] = a.d8[base + i];
#pragma unroll
        for (int i = 0; i < IPT; ++i) dk[i] = db[i];
        if (FG) {
            const double2 *wp = reinterpret_cast<const double2 *>(a.w_comp + base);
            const double2 *gp = reinterpret_cast<const double2 *>(a.g_end + base);
#pragma unroll
            for (int q = 0; q < IPT / 2; ++q) {
                const double2 v = wp[q];
                wv[2 * q] = v.x;
                wv[2 * q + 1] = v.y;
                const double2 u = gp[q];
                gv[2 * q] = u.x;
                gv[2 * q + 1] = u.y;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int64_t k = base + i;
            const bool ok = k < a.n;
            ev[i] = ok ? a.e[k] : 0.0;
            dk[i] = ok ? (int)a.d8[k] : 0;
            if (FG) {
                wv[i] = ok ? a.w_comp[k] : 0.0;
                gv[i] = ok ? a.g_end[k] : 1.0;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i)
        if (dk[i] == 255) dk[i] = a.d32[base + i];
    __syncthreads();
    const uint64_t ep0 = s_ep0;

    for (int32_t j = a.j_begin; j < a.j_end; ++j) {
        const uint64_t ep = ep0 + (uint64_t)(j - a.j_begin);

        // ---- column j and the pending step of column j-1 into LDS
        {
            uint32_t *f32 = reinterpret_cast<uint32_t *>(s_flag);
            for (int i = tid; i < S / 4; i += BLOCK) f32[i] = 0u;
        }
        __syncthreads();
        const ColTile cj = col_tile(a.col, j, chunk0, chunk1);
        for (int32_t o = cj.lo + tid; o < cj.hi; o += BLOCK) {
            const int32_t r = (int32_t)(a.col.rows[cj.cb + o] - seg0);
            if (VALS) s_xv[r] = a.col.vals[cj.cb + o];
            lds_flag_or(s_flag, r, kFlagX);
        }
        if (j > a.j_begin) {
            if (tid == 0) {
                if (wait_flag(a.ws.sflags + b, ((ep - 1) << 1) | 1u, hdr)) {
                    order_acquire();
                    s_step = ld_relaxed(a.steps + (j - 1));
                } else {
                    s_abort = 1;
                }
            }
            __syncthreads();
            if (s_abort) return;
            const double st = s_step;
            if (st != 0.0) {
                const ColTile cp = col_tile(a.col, j - 1, chunk0, chunk1);
                for (int32_t o = cp.lo + tid; o < cp.hi; o += BLOCK) {
                    const int32_t k = a.col.rows[cp.cb + o];
                    const double x = VALS ? a.col.vals[cp.cb + o] : 1.0;
                    const double et = a.eta[k] + x * st;
                    const double en = exp(et);
                    a.eta[k] = et;
                    a.e[k] = en;
                    s_ep[k - seg0] = en;
                    lds_flag_or(s_flag, (int32_t)(k - seg0), kFlagPatch);
                }
            }
        }
        __syncthreads();
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

        // ---- tuple totals of the thread, block scan, segment aggregate
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
        double incl[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) incl[c] = run[c];
        wave_inclusive_scan<NC>(incl);
        if (lane == kWave - 1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) s_wsum[w][c] = incl[c];
        }
        __syncthreads();
        double texcl[NC];
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

        // ---- exchange 1: every segment aggregate to every workgroup
        if (tid == 0) {
            TileState *ts = a.ws.tiles + b;
#pragma unroll
            for (int c = 0; c < NC; ++c) st_relaxed(ts->agg + c, agg[c]);
            order_release();
            st_flag(&ts->flag, (ep << 2) | kStateAgg);
        }
        double pre[NC];
        double tot[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NC; ++c) pre[c] = 0.0;
        int bad = 0;
        for (int q = tid; q < G; q += BLOCK) {
            const TileState *ts = a.ws.tiles + q;
            if (!wait_flag(&ts->flag, (ep << 2) | kStateAgg, hdr)) {
                bad = 1;
                break;
            }
            order_acquire();
            double v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = ld_relaxed(ts->agg + c);
            if (q < b) {
#pragma unroll
                for (int c = 0; c < NC; ++c) pre[c] += v[c];
            }
            if (FG) {
#pragma unroll
                for (int c = 0; c < 3; ++c) tot[c] += v[3 + c];
            }
        }
        if (__syncthreads_or(bad)) return;
        {
            double red[NC + 3];
#pragma unroll
            for (int c = 0; c < NC; ++c) red[c] = pre[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) red[NC + c] = tot[c];
            block_sum<NC + 3, BLOCK>(red, s_red);
            if (tid == 0) {
#pragma unroll
                for (int c = 0; c < NC + 3; ++c) s_bc[c] = red[c];
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < NC; ++c) texcl[c] += s_bc[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) tot[c] = s_bc[NC + c];
        }

        // ---- running prefix, transform at run ends, reduction
        double acc[3] = {0.0, 0.0, 0.0};
        double Sr[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) Sr[c] = texcl[c];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const double ex = ev[i] * xv[i];
            Sr[0] += ev[i];
            Sr[1] += ex;
            Sr[2] += ex * xv[i];
            if (FG) {
                const double ew = ev[i] * wv[i];
                const double exw = ew * xv[i];
                Sr[3] += ew;
                Sr[4] += exw;
                Sr[5] += exw * xv[i];
            }
            const int d = dk[i];
            if (d != 0) {
                double S0 = Sr[0], S1 = Sr[1], S2 = Sr[2];
                if (FG) {
                    const double g = gv[i];
                    S0 += g * (tot[0] - Sr[3]);
                    S1 += g * (tot[1] - Sr[4]);
                    S2 += g * (tot[2] - Sr[5]);
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
        block_sum<3, BLOCK>(acc, s_red);

        // ---- exchange 2: partials to workgroup 0, step back to everyone
        const uint64_t ptag = (ep << 1) | 1u;
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) st_relaxed(a.ws.partials + 4 * b + c, acc[c]);
            order_release();
            st_flag(a.ws.pflags + b, ptag);
        }
        if (b == 0) {
            double sum[3] = {0.0, 0.0, 0.0};
            bad = 0;
            for (int q = tid; q < G; q += BLOCK) {
                if (!wait_flag(a.ws.pflags + q, ptag, hdr)) {
                    bad = 1;
                    break;
                }
                order_acquire();
#pragma unroll
                for (int c = 0; c < 3; ++c) sum[c] += ld_relaxed(a.ws.partials + 4 * q + c);
            }
            if (__syncthreads_or(bad)) return;
            block_sum<3, BLOCK>(sum, s_red);
            if (tid == 0) {
                const double g1 = a.c[j] - sum[0];
                const double g2 = -sum[1];
                double bj = a.beta[j], dj = a.delta[j], st = 0.0;
                ccd_apply(g1, g2, a.penalty, a.lambda, &bj, &dj, &st);
                a.beta[j] = bj;
                a.delta[j] = dj;
                st_relaxed(a.steps + j, st);
                if (a.g12_out) {
                    a.g12_out[3 * j] = g1;
                    a.g12_out[3 * j + 1] = g2;
                    a.g12_out[3 * j + 2] = sum[2];
                }
                order_release();
            }
            __syncthreads();
            for (int q = tid; q < G; q += BLOCK) st_flag(a.ws.sflags + q, ptag);
        }
    }

    // ---- the last coordinate's update of eta and e
    const int32_t jl = a.j_end - 1;
    const uint64_t ep_last = ep0 + (uint64_t)(jl - a.j_begin);
    if (tid == 0) {
        if (wait_flag(a.ws.sflags + b, (ep_last << 1) | 1u, hdr)) {
            order_acquire();
            s_step = ld_relaxed(a.steps + jl);
        } else {
            s_abort = 1;
        }
    }
    __syncthreads();
    if (s_abort) return;
    const double st = s_step;
    if (st != 0.0) {
        const ColTile cp = col_tile(a.col, jl, chunk0, chunk1);
        for (int32_t o = cp.lo + tid; o < cp.hi; o += BLOCK) {
            const int32_t k = a.col.rows[cp.cb + o];
            const double x = VALS ? a.col.vals[cp.cb + o] : 1.0;
            const double et = a.eta[k] + x * st;
            a.eta[k] = et;
            a.e[k] = exp(et);
        }
    }
    // every workgroup read the epoch before exchange 1 of the first
    // coordinate, which workgroup 0 waited for
    if (b == 0 && tid == 0)
        st_relaxed_u64(&hdr->epoch, ep0 + (uint64_t)(a.j_end - a.j_begin));
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

template <int BLOCK, int IPT>
void *pick_kernel(int model, bool vals)
{
    if (model == SS_FINE_GRAY)
        return vals ? kernel_ptr<BLOCK, IPT, SS_FINE_GRAY, true>()
                    : kernel_ptr<BLOCK, IPT, SS_FINE_GRAY, false>();
    return vals ? kernel_ptr<BLOCK, IPT, SS_COX, true>() : kernel_ptr<BLOCK, IPT, SS_COX, false>();
}

void *kernel_for(int block, int ipt, int model, bool vals)
{
    if (block == 512 && ipt == 4) return pick_kernel<512, 4>(model, vals);
    if (block == 512 && ipt == 8) return pick_kernel<512, 8>(model, vals);
    if (block == 512 && ipt == 16) return pick_kernel<512, 16>(model, vals);
    return nullptr;
}

}  // namespace

int32_t launch_sweep_persistent(const SweepCall &call, const WsView &ws, hipStream_t s)
{
    // segments of 2048, 4096 or 8192 positions; LDS holds a segment's flags,
    // column values and patched e (8192 positions: 136 KB of 160 KB)
    static const Shape shapes[] = {{512, 4}, {512, 8}, {512, 16}};
    int dev = 0;
    SS_HIP_CHECK(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    SS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SS_HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return SS_EUNSUPPORTED;
    const bool vals = call.col.vals != nullptr;
    for (const Shape &sh : shapes) {
        const int64_t seg = (int64_t)sh.block * sh.ipt;
        const int64_t G = ceil_div(call.n, seg);
        // a few hundred segments at most: the all-to-all exchange reads G
        // aggregates per workgroup
        if (G > 512 || G > ws.max_tiles) continue;
        void *k = kernel_for(sh.block, sh.ipt, call.model, vals);
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
