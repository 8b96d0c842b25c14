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
// around element-wise passes in sorted order; the gradient reaches subject
// order by one gather through the inverse permutation.  l is a sum of fixed-grid block
// partials; every sum is taken in a fixed order.
#include <math.h>

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

// At run ends: q = d / S0, q2 = d G / S0 (Fine-Gray); the likelihood terms
// delta eta - d log S0 summed per block (fixed grid, fixed order) into
// lpart[blockIdx].
constexpr int kAdjGrid = 2048;

__global__ __launch_bounds__(256) void k_adj_terms(int32_t model, int64_t n,
                                                   const int8_t *status_s, const double *eta,
                                                   const uint8_t *d8, const int32_t *d32,
                                                   const double *g_end, const double *p0,
                                                   const double *pw, double *q, double *q2,
                                                   double *lpart)
{
    __shared__ double s_red[4];
    const bool fg = model == SS_FINE_GRAY;
    const double tot_w = fg ? pw[n - 1] : 0.0;
    double lsum = 0.0;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        int d = d8[k];
        if (d == 255) d = d32[k];
        double l = is_event(model, status_s[k]) ? eta[k] : 0.0;
        double qk = 0.0, q2k = 0.0;
        if (d != 0) {
            double s0 = p0[k];
            if (fg) s0 += g_end[k] * (tot_w - pw[k]);
            qk = (double)d / s0;
            if (fg) q2k = (double)d * g_end[k] / s0;
            l -= (double)d * log(s0);
        }
        q[k] = qk;
        if (fg) q2[k] = q2k;
        lsum += l;
    }
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_down(lsum, o);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) lpart[blockIdx.x] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

// dl/deta in sorted order (coalesced); block 0 adds the likelihood
// partials in order.
__global__ __launch_bounds__(256) void k_adj_grad(int32_t model, int64_t n,
                                                  const int8_t *status_s, const double *e,
                                                  const double *w_comp, const double *r,
                                                  const double *q2x, const double *lpart,
                                                  int nlpart, double *grad_s, double *loglik)
{
    const bool fg = model == SS_FINE_GRAY;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        double inner = r[k];
        if (fg) inner += w_comp[k] * q2x[k];
        grad_s[k] = (is_event(model, status_s[k]) ? 1.0 : 0.0) - e[k] * inner;
    }
    if (blockIdx.x == 0) {
        __shared__ double s_red[4];
        double l = 0.0;
        for (int b = threadIdx.x; b < nlpart; b += 256) l += lpart[b];
        for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = l;
        __syncthreads();
        if (threadIdx.x == 0) *loglik = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
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
    t.lpart = (double *)take(8 * (size_t)kAdjGrid);
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

int32_t launch_eta_gradient(int32_t model, int64_t n, const int32_t *inv_perm,
                            const int8_t *status_s, const double *eta, const double *e,
                            const uint8_t *d8, const int32_t *d32, const double *w_comp,
                            const double *g_end, double *grad, double *loglik, void *ws,
                            hipStream_t s)
{
    AdjWs w;
    adj_layout(n, ws, &w);
    const bool fg = model == SS_FINE_GRAY;
    const int grid = grid_of(n);
    int32_t rc = scan_add_f64(e, w.a, n, false, false, w.sums, s);  // prefix of e
    if (rc) return rc;
    if (fg) {
        hipLaunchKernelGGL(k_adj_mul, dim3(grid), dim3(256), 0, s, n, e, w_comp, w.b);
        SS_LAUNCH_CHECK();
        rc = scan_add_f64(w.b, w.b, n, false, false, w.sums, s);      // prefix of e w
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_adj_terms, dim3(grid), dim3(256), 0, s, model, n, status_s, eta, d8,
                       d32, g_end, w.a, w.b, w.q, w.q2, w.lpart);
    SS_LAUNCH_CHECK();
    rc = scan_add_f64(w.q, w.a, n, true, false, w.sums, s);           // suffix of d / S0
    if (rc) return rc;
    if (fg) {
        rc = scan_add_f64(w.q2, w.b, n, false, true, w.sums, s);      // run ends before k
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_adj_grad, dim3(grid), dim3(256), 0, s, model, n, status_s, e, w_comp,
                       w.a, w.b, w.lpart, grid, w.q, loglik);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_adj_to_subjects, dim3(grid), dim3(256), 0, s, n, inv_perm, w.q, grad);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace ss
