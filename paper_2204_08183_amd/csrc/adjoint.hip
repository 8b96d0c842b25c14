// The full gradient of the log (pseudo-)likelihood with respect to eta, for
// every subject, in O(N) (the vector delta - P delta of Sec. 2.9, which a
// proximal-gradient step multiplies by X'; Sec. 2.9 notes the prefix-sum
// form of Sec. 2.7 applies).  With the subjects by decreasing time and d_k
// the events of the tie run ending at k (Breslow):
//
//   S0_k   = prefix(e)_k [+ G(Y_k) * (sum of e w after k's run), Fine-Gray]
//   dl/deta_m = delta_m - e_m * ( sum_{run ends k >= m} d_k / S0_k
//               [+ w_m * sum_{run ends k < m} d_k G(Y_k) / S0_k, Fine-Gray] )
//   l      = sum_m delta_m eta_m - sum_k d_k log S0_k
//
// with w = I(status = 2) / G(y) the competing-event weight.  Scans (prefix
// of e, suffix of d/S0, and for Fine-Gray the prefix of e w and of d G/S0)
// in sorted order, the run-end terms computed in the last pass of the scan
// of e and the gradient in the last pass of the suffix scan of d/S0; the
// gradient reaches subject order by one gather through the inverse
// permutation.  l is a sum of per-tile partials; every sum is taken in a
// fixed order.
#include <math.h>

#include "scan_device.h"
#include "ss_internal.h"

namespace ss {

namespace {

__device__ __forceinline__ bool is_event(int32_t model, int8_t s)
{
    return model == SS_FINE_GRAY ? s == 1 : s != 0;
}

__global__ __launch_bounds__(256) void k_adj_mul(int64_t n, const double *a, const double *b,
                                                 double *out)
{
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        out[k] = a[k] * b[k];
}

constexpr int kAdjGrid = 2048;  // workgroups of the element-wise passes

// Eight consecutive bytes of a thread's scan items (memory order).
__device__ __forceinline__ void load_bytes8(const uint8_t *p, int64_t k0, int64_t n,
                                            uint8_t (&b)[SI])
{
    if (k0 + SI <= n && ((uintptr_t)(p + k0) & 7u) == 0) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p + k0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b[i] = (uint8_t)(v.x >> (8 * i));
            b[4 + i] = (uint8_t)(v.y >> (8 * i));
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < SI; ++i) b[i] = k0 + i < n ? p[k0 + i] : 0;
}

// Fixed-order sum of one value per thread of the workgroup; thread 0 gets it.
__device__ __forceinline__ double block_total(double v, double *s_red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

// Last pass of the prefix scan of e, with the run-end terms: S0 at k is the
// prefix (Fine-Gray: plus G(Y_k) times the e w after k, from pw), q = d/S0,
// q2 = d G/S0, and the tile's sum of delta eta - d log S0 into lpart[tile].
template <bool FG>
__global__ __launch_bounds__(SB) void k_adj_scan_terms(int64_t n, const double *e,
                                                       const double *carry,
                                                       const int8_t *status_s,
                                                       const double *eta, const uint8_t *d8,
                                                       const int32_t *d32, const double *g_end,
                                                       const double *pw, double *q,
                                                       double *q2, double *lpart)
{
    static_assert(SB == 4 * kWave, "block_total sums four waves");
    __shared__ double s_w[SB / kWave];
    __shared__ double s_red[SB / kWave];
    const int64_t k0 = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    double s0[SI], et[SI];
    load_items<double, OpAdd<double>, false>(e, k0, n, s0);
    block_scan<double, OpAdd<double>>(s0, carry[blockIdx.x], s_w);
    load_items<double, OpAdd<double>, false>(eta, k0, n, et);
    uint8_t dd[SI], st[SI];
    load_bytes8(d8, k0, n, dd);
    load_bytes8(reinterpret_cast<const uint8_t *>(status_s), k0, n, st);
    const double tot_w = FG ? pw[n - 1] : 0.0;
    double qv[SI], q2v[SI];
    double lsum = 0.0;
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int64_t k = k0 + i;
        qv[i] = 0.0;
        q2v[i] = 0.0;
        if (k < n) {
            int d = dd[i];
            if (d == 255) d = d32[k];
            double l = is_event(FG ? SS_FINE_GRAY : SS_COX, (int8_t)st[i]) ? et[i] : 0.0;
            if (d != 0) {
                double S0 = s0[i];
                double g = 0.0;
                if (FG) {
                    g = g_end[k];
                    S0 += g * (tot_w - pw[k]);
                }
                qv[i] = (double)d / S0;
                if (FG) q2v[i] = (double)d * g / S0;
                l -= (double)d * log(S0);
            }
            lsum += l;
        }
    }
    store_items<double, false>(q, k0, n, qv);
    if (FG) store_items<double, false>(q2, k0, n, q2v);
    const double t = block_total(lsum, s_red);
    if (threadIdx.x == 0) lpart[blockIdx.x] = t;
}

// Last pass of the suffix scan of q = d/S0: R at k is the suffix, and
// dl/deta_k = delta_k - e_k (R + w_k Q_k) (Q: the exclusive prefix of
// q2, Fine-Gray) goes to grad_s in sorted order.  Workgroup 0 also adds
// the likelihood partials in order.
template <bool FG>
__global__ __launch_bounds__(SB) void k_adj_scan_grad(int64_t n, const double *q,
                                                      const double *carry,
                                                      const int8_t *status_s, const double *e,
                                                      const double *w_comp, const double *q2x,
                                                      const double *lpart, int64_t nlpart,
                                                      double *grad_s, double *loglik)
{
    __shared__ double s_w[SB / kWave];
    __shared__ double s_red[SB / kWave];
    // scan position l holds sorted position n - 1 - l; a thread's items are
    // the descending run of sorted positions n - 1 - l0 .. n - SI - l0
    const int64_t l0 = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    double r[SI], ev[SI], wq[SI];
    load_items<double, OpAdd<double>, true>(q, l0, n, r);
    block_scan<double, OpAdd<double>>(r, carry[blockIdx.x], s_w);
    load_items<double, OpAdd<double>, true>(e, l0, n, ev);
    if (FG) {
        double wv[SI], qx[SI];
        load_items<double, OpAdd<double>, true>(w_comp, l0, n, wv);
        load_items<double, OpAdd<double>, true>(q2x, l0, n, qx);
#pragma unroll
        for (int i = 0; i < SI; ++i) wq[i] = wv[i] * qx[i];
    }
    double gv[SI];
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int64_t l = l0 + i;
        double inner = r[i];
        if (FG) inner += wq[i];
        const bool ev_k = l < n && is_event(FG ? SS_FINE_GRAY : SS_COX, status_s[n - 1 - l]);
        gv[i] = (ev_k ? 1.0 : 0.0) - ev[i] * inner;
    }
    store_items<double, true>(grad_s, l0, n, gv);
    if (blockIdx.x == 0) {
        double v = 0.0;
        for (int64_t b = threadIdx.x; b < nlpart; b += SB) v += lpart[b];
        const double t = block_total(v, s_red);
        if (threadIdx.x == 0) *loglik = t;
    }
}

// Subject order: a gather through the inverse permutation (random reads
// cost less than random partial-line writes).
__global__ __launch_bounds__(256) void k_adj_to_subjects(int64_t n, const int32_t *inv_perm,
                                                         const double *grad_s, double *grad)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        grad[i] = grad_s[inv_perm[i]];
}

// X' g over the sorted-position CSC design, cut along the positions into
// spans of kspan chunks (kspan * SS_CHUNK positions): one wave sums column
// j's non-zeros inside span c, found through the chunk index, into
// part[j * nspan + c].  A wave's unit is (span, column group); the waves of
// one span sit next to each other in launch order, so the stretch of g a
// span gathers from stays in L2 while its columns are summed.  Every sum is
// in a fixed order (four interleaved accumulators, then the wave), so the
// result is deterministic.
constexpr int kXtWaves = 4;

__global__ __launch_bounds__(256) void k_xt_span(int64_t p, int64_t nspan, int64_t kspan,
                                                 int64_t nchunk, int64_t groups,
                                                 const int64_t *col_ptr,
                                                 const int32_t *chunk_ptr,
                                                 const int32_t *rows_sorted,
                                                 const double *vals_sorted, const double *g,
                                                 double *part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t unit = (int64_t)blockIdx.x * kXtWaves + (threadIdx.x >> 6);
    if (unit >= nspan * groups) return;  // the whole wave
    const int64_t c = unit / groups;
    const int64_t t0 = c * kspan, t1 = min(t0 + kspan, nchunk);
    for (int64_t j = unit - c * groups; j < p; j += groups) {
        const int32_t *cp = chunk_ptr + j * (nchunk + 1);
        const int64_t base = col_ptr[j];
        const int64_t hi = base + cp[t1];
        int64_t q = base + cp[t0] + lane;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (vals_sorted) {
            for (; q + 3 * kWave < hi; q += 4 * kWave) {
                a0 += vals_sorted[q] * g[rows_sorted[q]];
                a1 += vals_sorted[q + kWave] * g[rows_sorted[q + kWave]];
                a2 += vals_sorted[q + 2 * kWave] * g[rows_sorted[q + 2 * kWave]];
                a3 += vals_sorted[q + 3 * kWave] * g[rows_sorted[q + 3 * kWave]];
            }
            for (; q < hi; q += kWave) a0 += vals_sorted[q] * g[rows_sorted[q]];
        } else {
            for (; q + 3 * kWave < hi; q += 4 * kWave) {
                a0 += g[rows_sorted[q]];
                a1 += g[rows_sorted[q + kWave]];
                a2 += g[rows_sorted[q + 2 * kWave]];
                a3 += g[rows_sorted[q + 3 * kWave]];
            }
            for (; q < hi; q += kWave) a0 += g[rows_sorted[q]];
        }
        const double v = dpp_wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) part[j * nspan + c] = v;
    }
}

// grad_beta[j] = the sum of column j's span partials, one workgroup per
// column: four interleaved accumulators per thread, then the workgroup's
// fixed-order sum.
__global__ __launch_bounds__(256) void k_xt_cols(int64_t nspan, const double *part, double *out)
{
    __shared__ double s_red[4];
    const double *pj = part + (int64_t)blockIdx.x * nspan;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t c = threadIdx.x;
    for (; c + 768 < nspan; c += 1024) {
        a0 += pj[c];
        a1 += pj[c + 256];
        a2 += pj[c + 512];
        a3 += pj[c + 768];
    }
    for (; c < nspan; c += 256) a0 += pj[c];
    const double t = block_total((a0 + a1) + (a2 + a3), s_red);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

struct AdjWs {
    double *a, *b, *q, *q2, *lpart;
    void *sums;
};

size_t adj_layout(int64_t n, void *ws, AdjWs *w)
{
    char *p = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *r = p ? p + off : nullptr;
        off = align_up(off + bytes, 256);
        return r;
    };
    AdjWs t;
    t.a = (double *)take(8 * (size_t)n);
    t.b = (double *)take(8 * (size_t)n);
    t.q = (double *)take(8 * (size_t)n);
    t.q2 = (double *)take(8 * (size_t)n);
    t.lpart = (double *)take(8 * (size_t)ceil_div(n, ST));
    t.sums = take(scan_sums_bytes(n));
    if (w) *w = t;
    return off;
}

int grid_of(int64_t n) { return (int)std::min<int64_t>(kAdjGrid, ceil_div(n, 256)); }

__global__ __launch_bounds__(256) void k_gather_u8(int64_t n, const int32_t *perm,
                                                   const uint8_t *src, uint8_t *dst)
{
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        dst[k] = src[perm[k]];
}

}  // namespace

int32_t launch_gather_u8(int64_t n, const int32_t *perm, const uint8_t *src, uint8_t *dst,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_u8, dim3(grid_of(n)), dim3(256), 0, s, n, perm, src, dst);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

size_t adjoint_ws_bytes(int64_t n) { return adj_layout(n, nullptr, nullptr); }

// The gradient in eta in sorted order into w.a (and l into *loglik).
static int32_t eta_gradient_sorted(int32_t model, int64_t n, const int8_t *status_s,
                                   const double *eta, const double *e, const uint8_t *d8,
                                   const int32_t *d32, const double *w_comp,
                                   const double *g_end, double *loglik, const AdjWs &w,
                                   hipStream_t s)
{
    const bool fg = model == SS_FINE_GRAY;
    const int grid = grid_of(n);
    const unsigned tiles = (unsigned)ceil_div(n, ST);
    const double *carry = reinterpret_cast<const double *>(w.sums);
    int32_t rc;
    if (fg) {
        hipLaunchKernelGGL(k_adj_mul, dim3(grid), dim3(256), 0, s, n, e, w_comp, w.b);
        SS_LAUNCH_CHECK();
        rc = scan_add_f64(w.b, w.b, n, false, false, w.sums, s);      // prefix of e w
        if (rc) return rc;
    }
    rc = scan_carries_f64(e, n, false, w.sums, s);                    // prefix of e, then
    if (rc) return rc;                                                 // the run-end terms
    if (fg) {
        hipLaunchKernelGGL(k_adj_scan_terms<true>, dim3(tiles), dim3(SB), 0, s, n, e, carry,
                           status_s, eta, d8, d32, g_end, w.b, w.q, w.q2, w.lpart);
    } else {
        hipLaunchKernelGGL(k_adj_scan_terms<false>, dim3(tiles), dim3(SB), 0, s, n, e, carry,
                           status_s, eta, d8, d32, g_end, w.b, w.q, w.q2, w.lpart);
    }
    SS_LAUNCH_CHECK();
    if (fg) {
        rc = scan_add_f64(w.q2, w.b, n, false, true, w.sums, s);      // run ends before k
        if (rc) return rc;
    }
    rc = scan_carries_f64(w.q, n, true, w.sums, s);                   // suffix of d / S0,
    if (rc) return rc;                                                 // then the gradient
    if (fg) {
        hipLaunchKernelGGL(k_adj_scan_grad<true>, dim3(tiles), dim3(SB), 0, s, n, w.q, carry,
                           status_s, e, w_comp, w.b, w.lpart, (int64_t)tiles, w.a, loglik);
    } else {
        hipLaunchKernelGGL(k_adj_scan_grad<false>, dim3(tiles), dim3(SB), 0, s, n, w.q, carry,
                           status_s, e, w_comp, w.b, w.lpart, (int64_t)tiles, w.a, loglik);
    }
    SS_LAUNCH_CHECK();
    return SS_OK;
}

int32_t launch_eta_gradient(int32_t model, int64_t n, const int32_t *inv_perm,
                            const int8_t *status_s, const double *eta, const double *e,
                            const uint8_t *d8, const int32_t *d32, const double *w_comp,
                            const double *g_end, double *grad, double *loglik, void *ws,
                            hipStream_t s)
{
    AdjWs w;
    adj_layout(n, ws, &w);
    const int32_t rc = eta_gradient_sorted(model, n, status_s, eta, e, d8, d32, w_comp, g_end,
                                           loglik, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_adj_to_subjects, dim3(grid_of(n)), dim3(256), 0, s, n, inv_perm, w.a,
                       grad);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

// Span length (in chunks) of the X' pass: 8 chunks (8192 positions), longer
// where p * spans would pass 2 (n + p) partials (designs much wider than
// long), which bounds the workspace.
int64_t xt_span_chunks(int64_t n, int64_t p)
{
    const int64_t nchunk = ceil_div(n, (int64_t)SS_CHUNK);
    int64_t k = 8;
    while (k < nchunk && p * ceil_div(nchunk, k) > 2 * (n + p)) k *= 2;
    return k;
}

size_t beta_ws_bytes(int64_t n, int64_t p)
{
    const int64_t nspan = ceil_div(ceil_div(n, (int64_t)SS_CHUNK), xt_span_chunks(n, p));
    return adjoint_ws_bytes(n) + align_up(8 * (size_t)p * (size_t)nspan, 256);
}

int32_t launch_beta_gradient(int32_t model, int64_t n, int64_t p, const int32_t *inv_perm,
                             const int8_t *status_s, const double *eta, const double *e,
                             const uint8_t *d8, const int32_t *d32, const double *w_comp,
                             const double *g_end, const int64_t *col_ptr,
                             const int32_t *rows_sorted, const double *vals_sorted,
                             const int32_t *chunk_ptr, double *grad_beta, double *grad_eta,
                             double *loglik, void *ws, hipStream_t s)
{
    AdjWs w;
    adj_layout(n, ws, &w);
    int32_t rc = eta_gradient_sorted(model, n, status_s, eta, e, d8, d32, w_comp, g_end, loglik,
                                     w, s);
    if (rc) return rc;
    const int64_t nchunk = ceil_div(n, (int64_t)SS_CHUNK);
    const int64_t kspan = xt_span_chunks(n, p);
    const int64_t nspan = ceil_div(nchunk, kspan);
    // about 16K waves when the design allows: column groups per span
    const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(p, ceil_div(16384, nspan)));
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + adjoint_ws_bytes(n));
    hipLaunchKernelGGL(k_xt_span, dim3((unsigned)ceil_div(nspan * groups, kXtWaves)), dim3(256),
                       0, s, p, nspan, kspan, nchunk, groups, col_ptr, chunk_ptr, rows_sorted,
                       vals_sorted, w.a, part);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_xt_cols, dim3((unsigned)p), dim3(256), 0, s, nspan, part, grad_beta);
    SS_LAUNCH_CHECK();
    if (grad_eta) {
        hipLaunchKernelGGL(k_adj_to_subjects, dim3(grid_of(n)), dim3(256), 0, s, n, inv_perm,
                           w.a, grad_eta);
        SS_LAUNCH_CHECK();
    }
    return SS_OK;
}

}  // namespace ss
