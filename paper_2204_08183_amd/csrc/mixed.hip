// FP32-storage path (e in FP32, three accumulation modes) for the Cox and
// Fine-Gray coordinate gradient and Hessian: the same quantities as the
// fused FP64 kernels (steps (2)-(4) of Sec. 2.7), computed with
//   SS_ACC_F32       plain FP32 sums,
//   SS_ACC_F32_COMP  compensated FP32 sums (hi + lo, two-sum),
//   SS_ACC_F64       FP64 sums of the FP32 inputs,
//   SS_ACC_F32_C64   FP32 sums inside a tile, FP64 across tiles: the
//                    carry between tiles (the prefix a tile starts from)
//                    and the sum of the tile partials are FP64, everything
//                    else (in-tile scan, transform, in-tile reduction) FP32,
// so that the error of each against the FP64 definition can be measured.
// Accuracy is the point here, so the scan is a plain reduce-then-scan in a
// fixed order: per-tile aggregates, one scan of them, then the tile pass
// with its transform and reduction, then the final sum.
//
// e is stored as exp(eta - m) with m = max eta (exp overflows FP32 from
// eta ~ 88): g' and g'' do not depend on the shift, and sum d log S0 moves
// by m sum d.
#include <math.h>

#include "ss_device.h"

namespace ss {

namespace {

using namespace dev;

constexpr int kMxBlock = 256;
constexpr int kMxIpt = 16;
constexpr int kMxTile = kMxBlock * kMxIpt;  // whole chunks of the column index
static_assert(kMxTile % SS_CHUNK == 0, "mixed tile must be whole chunks");

// ---------------------------------------------------------------- accumulators
// Knuth's two-sum: s + t == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &t)
{
    s = a + b;
    const float bb = s - a;
    t = (a - (s - bb)) + (b - bb);
}

template <int ACC>
struct Acc;

template <>
struct Acc<SS_ACC_F32> {
    typedef float T;
    float s;  // no initialiser: the type lives in LDS arrays too; see zero()
    __device__ void zero() { s = 0.f; }
    __device__ void add(float x) { s += x; }
    __device__ void merge(const Acc &o) { s += o.s; }
    __device__ float value() const { return s; }
    __device__ double hi() const { return s; }
    __device__ double lo() const { return 0.0; }
    __device__ void set(double h, double) { s = (float)h; }
};

template <>
struct Acc<SS_ACC_F32_COMP> {
    typedef float T;
    float h, l;
    __device__ void zero() { h = l = 0.f; }
    __device__ void add(float x)
    {
        float s, t;
        two_sum(h, x, s, t);
        h = s;
        l += t;
    }
    __device__ void merge(const Acc &o)
    {
        float s, t;
        two_sum(h, o.h, s, t);
        h = s;
        l += o.l + t;
    }
    __device__ float value() const { return h + l; }
    __device__ double hi() const { return h; }
    __device__ double lo() const { return l; }
    __device__ void set(double a, double b)
    {
        h = (float)a;
        l = (float)b;
    }
};

template <>
struct Acc<SS_ACC_F64> {
    typedef double T;
    double s;
    __device__ void zero() { s = 0.0; }
    __device__ void add(double x) { s += x; }
    __device__ void merge(const Acc &o) { s += o.s; }
    __device__ double value() const { return s; }
    __device__ double hi() const { return s; }
    __device__ double lo() const { return 0.0; }
    __device__ void set(double h, double) { s = h; }
};

// FP32 inside a tile, FP64 across tiles: `c` holds what came from other
// tiles (set() from a stored prefix or partial, merges of such values), `s`
// what was summed inside this tile.  Tile aggregates and partials leave a
// tile as c + s and are merged in FP64; the running prefix of the tile pass
// is the FP64 carry plus the FP32 in-tile sum.
template <>
struct Acc<SS_ACC_F32_C64> {
    typedef float T;
    double c;
    float s;
    __device__ void zero()
    {
        c = 0.0;
        s = 0.f;
    }
    __device__ void add(float x) { s += x; }
    __device__ void merge(const Acc &o)
    {
        c += o.c;
        s += o.s;
    }
    __device__ double value() const { return c + (double)s; }
    __device__ double hi() const { return c + (double)s; }
    __device__ double lo() const { return 0.0; }
    __device__ void set(double h, double l)
    {
        c = h + l;
        s = 0.f;
    }
};

// Inclusive block scan (Hillis-Steele in LDS, fixed order) of NC
// accumulators per thread; also returns the block total in every thread.
template <int ACC, int NC>
__device__ void block_scan(Acc<ACC> (&x)[NC], Acc<ACC> (&total)[NC], Acc<ACC> *s_buf)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NC; ++c) s_buf[c * kMxBlock + tid] = x[c];
    __syncthreads();
    for (int off = 1; off < kMxBlock; off <<= 1) {
        Acc<ACC> y[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            y[c] = s_buf[c * kMxBlock + tid];
            if (tid >= off) {
                Acc<ACC> lhs = s_buf[c * kMxBlock + tid - off];
                lhs.merge(y[c]);
                y[c] = lhs;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) s_buf[c * kMxBlock + tid] = y[c];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        x[c] = s_buf[c * kMxBlock + tid];
        total[c] = s_buf[c * kMxBlock + kMxBlock - 1];
    }
    __syncthreads();
}

struct MixedCall {
    int32_t model;
    int64_t n;
    int64_t p;
    int32_t j;
    const float *e;
    const uint8_t *d8;
    const int32_t *d32;
    const double *w_comp;
    const double *g_end;
    Column col;
    const double *c;
    double *out;
};

// Tile data in the accumulation type: e (and e w), x of column j, d.
template <int ACC, bool FG>
__device__ void load_tile(const MixedCall &a, int64_t t0, typename Acc<ACC>::T (&ev)[kMxIpt],
                          typename Acc<ACC>::T (&wv)[FG ? kMxIpt : 1],
                          typename Acc<ACC>::T (&xv)[kMxIpt], int (&dk)[kMxIpt],
                          typename Acc<ACC>::T *s_x, uint8_t *s_nz)
{
    typedef typename Acc<ACC>::T T;
    const int tid = threadIdx.x;
    for (int i = tid; i < kMxTile; i += kMxBlock) s_nz[i] = 0;
    __syncthreads();
    const int64_t nchunk = a.col.nchunk1 - 1;
    const int64_t chunk0 = t0 / SS_CHUNK;
    const int64_t chunk1 = min(chunk0 + kMxTile / SS_CHUNK, nchunk);
    const ColTile ct = col_tile(a.col, a.j, chunk0, chunk1);
    for (int32_t o = ct.lo + tid; o < ct.hi; o += kMxBlock) {
        const int32_t r = (int32_t)(a.col.rows[ct.cb + o] - t0);
        s_x[r] = a.col.vals ? (T)a.col.vals[ct.cb + o] : (T)1;
        s_nz[r] = 1;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMxIpt; ++i) {
        const int r = tid * kMxIpt + i;
        const int64_t k = t0 + r;
        const bool ok = k < a.n;
        ev[i] = ok ? (T)a.e[k] : (T)0;
        if (FG) wv[FG ? i : 0] = ok ? (T)a.w_comp[k] : (T)0;
        xv[i] = s_nz[r] ? s_x[r] : (T)0;
        int d = ok ? (int)a.d8[k] : 0;
        if (d == 255) d = a.d32[k];
        dk[i] = d;
    }
}

// Components of the tuple at one position: (e, e x, e x^2) and, for
// Fine-Gray, (e w, e w x, e w x^2).
template <typename T, bool FG>
__device__ __forceinline__ void tuple_of(T e, T w, T x, T (&v)[FG ? 6 : 3])
{
    const T ex = e * x;
    v[0] = e;
    v[1] = ex;
    v[2] = ex * x;
    if (FG) {
        const T ew = e * w;
        const T exw = ew * x;
        v[3] = ew;
        v[4] = exw;
        v[5] = exw * x;
    }
}

// (1) Per-tile aggregates of the tuple, as (hi, lo) doubles in lb.
template <int ACC, bool FG>
__global__ __launch_bounds__(kMxBlock) void k_mx_tiles(MixedCall a, WsView ws)
{
    typedef typename Acc<ACC>::T T;
    constexpr int NC = FG ? 6 : 3;
    __shared__ T s_x[kMxTile];
    __shared__ uint8_t s_nz[kMxTile];
    __shared__ Acc<ACC> s_buf[NC * kMxBlock];
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * kMxTile;
    T ev[kMxIpt], wv[FG ? kMxIpt : 1], xv[kMxIpt];
    int dk[kMxIpt];
    load_tile<ACC, FG>(a, t0, ev, wv, xv, dk, s_x, s_nz);
    Acc<ACC> run[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) run[c].zero();
#pragma unroll
    for (int i = 0; i < kMxIpt; ++i) {
        T v[NC];
        tuple_of<T, FG>(ev[i], FG ? wv[FG ? i : 0] : (T)0, xv[i], v);
#pragma unroll
        for (int c = 0; c < NC; ++c) run[c].add(v[c]);
    }
    Acc<ACC> tot[NC];
    block_scan<ACC, NC>(run, tot, s_buf);
    if (threadIdx.x == 0) {
        double *dst = reinterpret_cast<double *>(ws.lb + tile * 8);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            dst[2 * c] = tot[c].hi();
            dst[2 * c + 1] = tot[c].lo();
        }
    }
}

// (2) Exclusive scan of the tile aggregates (one workgroup, fixed order),
// in place; Fine-Gray totals of the weighted components to the header.
template <int ACC, bool FG>
__global__ __launch_bounds__(kMxBlock) void k_mx_scan(WsView ws, int64_t ntiles)
{
    constexpr int NC = FG ? 6 : 3;
    __shared__ Acc<ACC> s_buf[NC * kMxBlock];
    const int tid = threadIdx.x;
    const int64_t per = (ntiles + kMxBlock - 1) / kMxBlock;
    const int64_t q0 = tid * per, q1 = min(q0 + per, ntiles);
    Acc<ACC> run[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) run[c].zero();
    for (int64_t q = q0; q < q1; ++q) {
        const double *src = reinterpret_cast<const double *>(ws.lb + q * 8);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Acc<ACC> t;
            t.set(src[2 * c], src[2 * c + 1]);
            run[c].merge(t);
        }
    }
    Acc<ACC> incl[NC], tot[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) incl[c] = run[c];
    block_scan<ACC, NC>(incl, tot, s_buf);
    // exclusive prefix of this thread's first tile: the inclusive scan of the
    // thread before (still in s_buf), then the thread's tiles in order
    // (inclusive minus own run would not be exact in floating point)
    Acc<ACC> pre[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) pre[c].zero();
    if (tid > 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) pre[c] = s_buf[c * kMxBlock + tid - 1];
    }
    __syncthreads();
    for (int64_t q = q0; q < q1; ++q) {
        double *slot = reinterpret_cast<double *>(ws.lb + q * 8);
        Acc<ACC> nxt[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Acc<ACC> t;
            t.set(slot[2 * c], slot[2 * c + 1]);
            nxt[c] = pre[c];
            nxt[c].merge(t);
            slot[2 * c] = pre[c].hi();
            slot[2 * c + 1] = pre[c].lo();
            pre[c] = nxt[c];
        }
    }
    if (FG && tid == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ws.hdr->fg_tot[c] = tot[3 + c].hi();
            ws.hdr->scratch_out[c] = tot[3 + c].lo();
        }
    }
}

// (3) Tile pass: in-tile scan from the tile's prefix, the transform at run
// ends and the reduction; per-tile (hi, lo) partials of A, B, L to part.
template <int ACC, bool FG>
__global__ __launch_bounds__(kMxBlock) void k_mx_transform(MixedCall a, WsView ws)
{
    typedef typename Acc<ACC>::T T;
    constexpr int NC = FG ? 6 : 3;
    __shared__ T s_x[kMxTile];
    __shared__ uint8_t s_nz[kMxTile];
    __shared__ Acc<ACC> s_buf[NC * kMxBlock];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * kMxTile;
    T ev[kMxIpt], wv[FG ? kMxIpt : 1], xv[kMxIpt];
    int dk[kMxIpt];
    load_tile<ACC, FG>(a, t0, ev, wv, xv, dk, s_x, s_nz);
    Acc<ACC> run[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) run[c].zero();
#pragma unroll
    for (int i = 0; i < kMxIpt; ++i) {
        T v[NC];
        tuple_of<T, FG>(ev[i], FG ? wv[FG ? i : 0] : (T)0, xv[i], v);
#pragma unroll
        for (int c = 0; c < NC; ++c) run[c].add(v[c]);
    }
    Acc<ACC> incl[NC], tot[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) incl[c] = run[c];
    block_scan<ACC, NC>(incl, tot, s_buf);
    // running prefix: tile prefix, then the threads before, then element by element
    Acc<ACC> S[NC];
    {
        const double *src = reinterpret_cast<const double *>(ws.lb + tile * 8);
#pragma unroll
        for (int c = 0; c < NC; ++c) S[c].set(src[2 * c], src[2 * c + 1]);
    }
    __syncthreads();
    // the exclusive prefix of this thread inside the tile, recomputed in the
    // fixed order: the inclusive scan of the thread before
#pragma unroll
    for (int c = 0; c < NC; ++c) s_buf[c * kMxBlock + tid] = incl[c];
    __syncthreads();
    if (tid > 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) S[c].merge(s_buf[c * kMxBlock + tid - 1]);
    }
    T totw[3] = {(T)0, (T)0, (T)0};
    if (FG) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Acc<ACC> t;
            t.set(ws.hdr->fg_tot[c], ws.hdr->scratch_out[c]);
            totw[c] = (T)t.value();
        }
    }
    Acc<ACC> A, B, L;
    A.zero();
    B.zero();
    L.zero();
#pragma unroll
    for (int i = 0; i < kMxIpt; ++i) {
        T v[NC];
        tuple_of<T, FG>(ev[i], FG ? wv[FG ? i : 0] : (T)0, xv[i], v);
#pragma unroll
        for (int c = 0; c < NC; ++c) S[c].add(v[c]);
        const int d = dk[i];
        if (d != 0) {
            T S0 = (T)S[0].value(), S1 = (T)S[1].value(), S2 = (T)S[2].value();
            if (FG) {
                const T g = (T)a.g_end[t0 + tid * kMxIpt + i];
                S0 += g * (totw[0] - (T)S[3].value());
                S1 += g * (totw[1] - (T)S[4].value());
                S2 += g * (totw[2] - (T)S[5].value());
            }
            const T G = S1 / S0;
            const T H = S2 / S0;
            const T dd = (T)d;
            A.add(dd * G);
            B.add(dd * (H - G * G));
            L.add(dd * (T)log(S0));
        }
    }
    __syncthreads();
    Acc<ACC> part[3] = {A, B, L}, ptot[3];
    block_scan<ACC, 3>(part, ptot, s_buf);
    if (tid == 0) {
        double *dst = reinterpret_cast<double *>(ws.part + tile * 4);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dst[2 * c] = ptot[c].hi();
            dst[2 * c + 1] = ptot[c].lo();
        }
    }
}

// (4) Sum of the tile partials (one workgroup, fixed order); g', g'', L.
template <int ACC>
__global__ __launch_bounds__(kMxBlock) void k_mx_final(MixedCall a, WsView ws, int64_t ntiles)
{
    __shared__ Acc<ACC> s_buf[3 * kMxBlock];
    const int tid = threadIdx.x;
    const int64_t per = (ntiles + kMxBlock - 1) / kMxBlock;
    const int64_t q0 = tid * per, q1 = min(q0 + per, ntiles);
    Acc<ACC> run[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) run[c].zero();
    for (int64_t q = q0; q < q1; ++q) {
        const double *src = reinterpret_cast<const double *>(ws.part + q * 4);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Acc<ACC> t;
            t.set(src[2 * c], src[2 * c + 1]);
            run[c].merge(t);
        }
    }
    Acc<ACC> tot[3];
    block_scan<ACC, 3>(run, tot, s_buf);
    if (tid == 0) {
        const double A = tot[0].hi() + tot[0].lo();
        const double B = tot[1].hi() + tot[1].lo();
        const double L = tot[2].hi() + tot[2].lo();
        a.out[0] = a.c[a.j] - A;
        a.out[1] = -B;
        a.out[2] = L;
    }
}

// e32 = (float) exp(eta - m), m = max eta: block maxima, then the maximum
// and the exponentials.
constexpr int kMaxBlocks = 1024;

__global__ __launch_bounds__(256) void k_mx_max_part(int64_t n, const double *eta, double *part)
{
    __shared__ double s[256];
    double m = -INFINITY;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        m = fmax(m, eta[k]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_mx_max_final(int nparts, const double *part,
                                                      double *shift)
{
    __shared__ double s[256];
    double m = -INFINITY;
    for (int i = threadIdx.x; i < nparts; i += 256) m = fmax(m, part[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *shift = s[0];
}

__global__ __launch_bounds__(256) void k_mx_exp(int64_t n, const double *eta, const double *shift,
                                                float *e32)
{
    const double m = *shift;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        e32[k] = (float)exp(eta[k] - m);
}

template <int ACC, bool FG>
int32_t launch_mixed_t(const MixedCall &a, const WsView &ws, hipStream_t s)
{
    const int64_t ntiles = ceil_div(a.n, kMxTile);
    hipLaunchKernelGGL((k_mx_tiles<ACC, FG>), dim3((unsigned)ntiles), dim3(kMxBlock), 0, s, a, ws);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mx_scan<ACC, FG>), dim3(1), dim3(kMxBlock), 0, s, ws, ntiles);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mx_transform<ACC, FG>), dim3((unsigned)ntiles), dim3(kMxBlock), 0, s, a,
                       ws);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mx_final<ACC>), dim3(1), dim3(kMxBlock), 0, s, a, ws, ntiles);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

template <int ACC>
int32_t launch_mixed_acc(const MixedCall &a, const WsView &ws, hipStream_t s)
{
    return a.model == SS_FINE_GRAY ? launch_mixed_t<ACC, true>(a, ws, s)
                                   : launch_mixed_t<ACC, false>(a, ws, s);
}

}  // namespace

int32_t launch_mixed(int32_t acc, int32_t model, int64_t n, int64_t p, int32_t j,
                     const float *e32, const uint8_t *d8, const int32_t *d32,
                     const double *w_comp, const double *g_end, const Column &col,
                     const double *c, double *out, const WsView &ws, hipStream_t s)
{
    MixedCall a;
    a.model = model;
    a.n = n;
    a.p = p;
    a.j = j;
    a.e = e32;
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    a.col = col;
    a.c = c;
    a.out = out;
    switch (acc) {
    case SS_ACC_F32: return launch_mixed_acc<SS_ACC_F32>(a, ws, s);
    case SS_ACC_F32_COMP: return launch_mixed_acc<SS_ACC_F32_COMP>(a, ws, s);
    case SS_ACC_F64: return launch_mixed_acc<SS_ACC_F64>(a, ws, s);
    case SS_ACC_F32_C64: return launch_mixed_acc<SS_ACC_F32_C64>(a, ws, s);
    default: return SS_EINVAL;
    }
}

int32_t launch_exp_f32(int64_t n, const double *eta, float *e32, double *shift,
                       const WsView &ws, hipStream_t s)
{
    const int nparts = (int)std::min<int64_t>(kMaxBlocks, ceil_div(n, 256));
    double *part = reinterpret_cast<double *>(ws.part);
    hipLaunchKernelGGL(k_mx_max_part, dim3(nparts), dim3(256), 0, s, n, eta, part);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mx_max_final, dim3(1), dim3(256), 0, s, nparts, part, shift);
    SS_LAUNCH_CHECK();
    const int grid = (int)std::min<int64_t>(2048, ceil_div(n, 256));
    hipLaunchKernelGGL(k_mx_exp, dim3(grid), dim3(256), 0, s, n, eta, shift, e32);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace ss
