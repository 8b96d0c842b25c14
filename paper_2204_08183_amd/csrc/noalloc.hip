// ss_grad_hess without a caller-supplied workspace, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid allocation).  The fused kernels' scratch (look-back
// pairs, per-tile partial sums, the launch counters) lives in one
// file-scope device array per GPU, sized for problems of up to
// SS_NOALLOC_MAX_N subjects.  Each device's copy has its own address, looked
// up once per device with hipGetSymbolAddress; the host never passes the
// array's own name to a kernel (on the host it is only a stand-in for the
// symbol).
#include <mutex>

#include "ss_internal.h"

namespace ss {
namespace {

constexpr size_t kScratchBytes = fused_ws_bytes(SS_NOALLOC_MAX_N);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of this device's scratch array.  The first call on a
// device looks it up and clears it (a fill kernel on `s`, ordered before
// the caller's launch on the same stream).
int32_t device_scratch(hipStream_t s, void **out)
{
    int dev = -1;
    SS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SS_EUNSUPPORTED;
    if (s) {
        hipDevice_t sdev = -1;
        SS_HIP_CHECK(hipStreamGetDevice(s, &sdev));
        if (sdev != dev) return SS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255u)) return SS_EDEVICE;
        const int32_t rc = launch_ws_init(p, kScratchBytes, s);
        if (rc != SS_OK) return rc;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SS_OK;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" {

size_t ss_noalloc_scratch_bytes(void) { return kScratchBytes; }

int32_t ss_grad_hess_noalloc(int32_t model, int64_t n, int64_t p, int64_t j,
                             const double *e, const uint8_t *d8, const int32_t *d32,
                             const double *w_comp, const double *g_end,
                             const int64_t *col_ptr, const int32_t *rows_sorted,
                             const double *vals_sorted, const int32_t *chunk_ptr,
                             const double *c, double *out, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (n < 1 || p < 1 || p > INT32_MAX || j < 0 || j >= p) return SS_EINVAL;
    if (n > SS_NOALLOC_MAX_N) return SS_EINVAL;
    if (!model_arrays_ok(model, e, d8, d32, w_comp, g_end)) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !out) return SS_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    const int32_t rc = device_scratch(s, &ws);
    if (rc != SS_OK) return rc;
    WsView v;
    if (!fused_ws_view(ws, kScratchBytes, n, &v)) return SS_EWORKSPACE;
    FusedCall a = {};
    a.model = model;
    a.n = n;
    a.p = p;
    a.j = (int32_t)j;
    a.jprev = -1;
    a.jnext = -1;
    a.e = const_cast<double *>(e);
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    a.col.col_ptr = col_ptr;
    a.col.rows = rows_sorted;
    a.col.vals = vals_sorted;
    a.col.chunk_ptr = chunk_ptr;
    a.col.nchunk1 = ss_chunk_count(n) + 1;
    a.c = c;
    a.out = out;
    a.want_log = 1;
    a.obj_penalty = -1;
    // the error word is shared with earlier calls: clear it, report it in out[3]
    a.clear_error = 1;
    a.err_out = out + 3;
    return launch_fused(a, v, s);
}

}  // extern "C"
