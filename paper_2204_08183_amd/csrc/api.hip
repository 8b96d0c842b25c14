// C ABI of libsurvscan (declared in include/survscan.h).  Every entry point
// validates its arguments on the host before launching anything and returns
// a status code; no exception crosses the interface.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ss_internal.h"

namespace ss {


static thread_local char g_last_hip[256] = "no HIP error recorded";

int32_t record_hip_error(hipError_t err)
{
    snprintf(g_last_hip, sizeof(g_last_hip), "HIP error %d: %s", (int)err,
             hipGetErrorString(err));
    return SS_EDEVICE;
}

static bool bad_size(int64_t n, int64_t p)
{
    return n < 1 || n > INT32_MAX || p < 1 || p > INT32_MAX;
}

static Column column(const int64_t *col_ptr, const int32_t *rows, const double *vals,
                     const int32_t *chunk_ptr, int64_t n);

// The whole sweep as one persistent launch (SS_EUNSUPPORTED when it does
// not fit on the device).
static int32_t sweep_persistent(int32_t model, int32_t penalty, double lambda, int64_t n,
                                int64_t j_begin, int64_t j_end, double *eta, double *e,
                                const uint8_t *d8, const int32_t *d32, const double *w_comp,
                                const double *g_end, const Column &col, const double *c,
                                double *beta, double *delta, double *steps, double *g12_out,
                                const WsView &v, hipStream_t s)
{
    SweepCall sc = {};
    sc.model = model;
    sc.n = n;
    sc.j_begin = (int32_t)j_begin;
    sc.j_end = (int32_t)j_end;
    sc.eta = eta;
    sc.e = e;
    sc.d8 = d8;
    sc.d32 = d32;
    sc.w_comp = w_comp;
    sc.g_end = g_end;
    sc.col = col;
    sc.c = c;
    sc.beta = beta;
    sc.delta = delta;
    sc.steps = steps;
    sc.g12_out = g12_out;
    sc.penalty = penalty;
    sc.lambda = lambda;
    return launch_sweep_persistent(sc, v, s);
}

// RAII helpers of the tuning calls.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
struct ForceScope {
    ForceScope(int32_t kind, int32_t choice) { tune_force() = TuneForce{kind, choice}; }
    ~ForceScope() { tune_force() = TuneForce{-1, 0}; }
};

static Column column(const int64_t *col_ptr, const int32_t *rows, const double *vals,
                     const int32_t *chunk_ptr, int64_t n)
{
    Column c;
    c.col_ptr = col_ptr;
    c.rows = rows;
    c.vals = vals;
    c.chunk_ptr = chunk_ptr;
    c.nchunk1 = ss_chunk_count(n) + 1;
    return c;
}

}  // namespace ss

using namespace ss;

extern "C" {

const char *ss_status_string(int32_t code)
{
    switch (code) {
    case SS_OK: return "ok";
    case SS_EINVAL: return "invalid argument or data";
    case SS_EWORKSPACE: return "workspace too small or not 256-byte aligned";
    case SS_EUNSUPPORTED: return "unsupported model or penalty";
    case SS_EDEVICE: return g_last_hip;
    default: return "unknown status";
    }
}

int64_t ss_chunk_count(int64_t n) { return n <= 0 ? 0 : ceil_div(n, SS_CHUNK); }

size_t ss_prepare_workspace_bytes(int64_t n, int64_t p, int64_t nnz)
{
    if (n < 1 || p < 1 || nnz < 0) return 0;
    return prepare_ws_bytes(n, p, nnz);
}

int32_t ss_prepare(int32_t model, int64_t n, int64_t p, int64_t nnz, const double *y,
                   const int8_t *status, const int64_t *col_ptr, const int32_t *rows,
                   const double *vals, int32_t *perm, int32_t *inv_perm, uint8_t *d8,
                   int32_t *d32, double *c, int32_t *rows_sorted, double *vals_sorted,
                   int32_t *chunk_ptr, double *w_comp, double *g_end, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (bad_size(n, p) || nnz < 0 || nnz > INT32_MAX) return SS_EINVAL;
    if (!y || !status || !col_ptr || !perm || !inv_perm || !d8 || !d32 || !c ||
        !chunk_ptr)
        return SS_EINVAL;
    if (nnz > 0 && (!rows || !rows_sorted)) return SS_EINVAL;
    if (vals && nnz > 0 && !vals_sorted) return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!w_comp || !g_end)) return SS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255u)) return SS_EWORKSPACE;
    if (ws_bytes < prepare_ws_bytes(n, p, nnz)) return SS_EWORKSPACE;
    return run_prepare(model, n, p, nnz, y, status, col_ptr, rows, vals, perm, inv_perm,
                       d8, d32, c, rows_sorted, vals_sorted, chunk_ptr, w_comp, g_end, ws,
                       ws_bytes, (hipStream_t)stream);
}

size_t ss_workspace_bytes(int32_t model, int64_t n)
{
    if ((model != SS_COX && model != SS_FINE_GRAY) || n < 1) return 0;
    return fused_ws_bytes(n);
}

int32_t ss_workspace_init(void *ws, size_t ws_bytes, void *stream)
{
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < sizeof(WsHeader)) return SS_EWORKSPACE;
    return launch_ws_init(ws, ws_bytes, (hipStream_t)stream);
}

int32_t ss_workspace_error(const void *ws, int32_t *flag, void *stream)
{
    if (!ws || !flag) return SS_EINVAL;
    uint32_t v = 0;
    const WsHeader *h = (const WsHeader *)ws;
    SS_HIP_CHECK(hipMemcpyAsync(&v, &h->error, sizeof(v), hipMemcpyDeviceToHost,
                                (hipStream_t)stream));
    SS_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    *flag = (int32_t)v;
    return SS_OK;
}

int32_t ss_grad_hess(int32_t model, int64_t n, int64_t p, int64_t j, const double *e,
                     const uint8_t *d8, const int32_t *d32, const double *w_comp,
                     const double *g_end, const int64_t *col_ptr,
                     const int32_t *rows_sorted, const double *vals_sorted,
                     const int32_t *chunk_ptr, const double *c, double *out, void *ws,
                     size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (bad_size(n, p) || j < 0 || j >= p) return SS_EINVAL;
    if (!model_arrays_ok(model, e, d8, d32, w_comp, g_end)) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !out) return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    FusedCall a = {};
    a.model = model;
    a.n = n;
    a.p = p;
    a.j = (int32_t)j;
    a.jprev = -1;
    a.e = const_cast<double *>(e);
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    a.col = column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n);
    a.c = c;
    a.out = out;
    a.want_log = 1;
    a.obj_penalty = -1;
    a.jnext = -1;
    return launch_fused(a, v, (hipStream_t)stream);
}

static int32_t loglik_call(int32_t model, int32_t penalty, double lambda, int64_t n,
                           int64_t p, const double *e, const uint8_t *d8, const int32_t *d32,
                           const double *w_comp, const double *g_end, const double *beta,
                           const double *c, double *out, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (bad_size(n, p)) return SS_EINVAL;
    if (!model_arrays_ok(model, e, d8, d32, w_comp, g_end)) return SS_EINVAL;
    if (!beta || !c || !out) return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    FusedCall a = {};
    a.model = model;
    a.n = n;
    a.p = p;
    a.j = -1;
    a.jprev = -1;
    a.e = const_cast<double *>(e);
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    // no column: the chunk range is empty, the tuple is (e, 0, 0)
    a.col.col_ptr = nullptr;
    a.col.rows = nullptr;
    a.col.vals = nullptr;
    a.col.chunk_ptr = nullptr;
    a.col.nchunk1 = ss_chunk_count(n) + 1;
    a.c = c;
    a.out = out;
    a.beta_ll = beta;
    a.want_log = 1;
    a.obj_penalty = penalty;
    a.obj_lambda = lambda;
    a.jnext = -1;
    return launch_fused(a, v, (hipStream_t)stream);
}

int32_t ss_loglik(int32_t model, int64_t n, int64_t p, const double *e, const uint8_t *d8,
                  const int32_t *d32, const double *w_comp, const double *g_end,
                  const double *beta, const double *c, double *out, void *ws,
                  size_t ws_bytes, void *stream)
{
    return loglik_call(model, -1, 0.0, n, p, e, d8, d32, w_comp, g_end, beta, c, out, ws,
                       ws_bytes, stream);
}

int32_t ss_objective(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                     const double *e, const uint8_t *d8, const int32_t *d32,
                     const double *w_comp, const double *g_end, const double *beta,
                     const double *c, double *out, void *ws, size_t ws_bytes, void *stream)
{
    if (penalty != SS_PENALTY_NONE && penalty != SS_PENALTY_L1 && penalty != SS_PENALTY_L2)
        return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && !(lambda > 0.0)) return SS_EINVAL;
    return loglik_call(model, penalty, lambda, n, p, e, d8, d32, w_comp, g_end, beta, c, out,
                       ws, ws_bytes, stream);
}

int32_t ss_ccd_update(int32_t penalty, double lambda, int64_t n, int64_t p, int64_t j,
                      const double *g12, double *beta, double *delta, double *step,
                      double *eta, double *e, const int64_t *col_ptr,
                      const int32_t *rows_sorted, const double *vals_sorted, void *stream)
{
    if (penalty != SS_PENALTY_NONE && penalty != SS_PENALTY_L1 && penalty != SS_PENALTY_L2)
        return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && !(lambda > 0.0)) return SS_EINVAL;
    if (bad_size(n, p) || j < 0 || j >= p) return SS_EINVAL;
    if (!g12 || !beta || !delta || !step || !eta || !e || !col_ptr || !rows_sorted)
        return SS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int32_t rc = launch_ccd_scalar(penalty, lambda, (int32_t)j, g12, beta, delta, step, s);
    if (rc) return rc;
    Column col = column(col_ptr, rows_sorted, vals_sorted, nullptr, n);
    return launch_apply(n, (int32_t)j, step, eta, e, col, s);
}

int32_t ss_ccd_sweep(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                     int64_t j_begin, int64_t j_end, double *eta, double *e,
                     const uint8_t *d8, const int32_t *d32, const double *w_comp,
                     const double *g_end, const int64_t *col_ptr,
                     const int32_t *rows_sorted, const double *vals_sorted,
                     const int32_t *chunk_ptr, const double *c, double *beta,
                     double *delta, double *steps, double *g12_out, void *ws,
                     size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && penalty != SS_PENALTY_L1 && penalty != SS_PENALTY_L2)
        return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && !(lambda > 0.0)) return SS_EINVAL;
    if (bad_size(n, p) || j_begin < 0 || j_end > p || j_begin > j_end) return SS_EINVAL;
    if (!model_arrays_ok(model, e, d8, d32, w_comp, g_end) || !eta) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !beta || !delta || !steps)
        return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    if (j_begin == j_end) return SS_OK;
    hipStream_t s = (hipStream_t)stream;
    // SURVSCAN_SWEEP=launch forces one launch per coordinate (comparison and
    // tests); by default the sweep is one cooperative launch when it fits.
    const char *mode = getenv("SURVSCAN_SWEEP");
    if (!(mode && strcmp(mode, "launch") == 0)) {
        const int32_t rc = sweep_persistent(
            model, penalty, lambda, n, j_begin, j_end, eta, e, d8, d32, w_comp, g_end,
            column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n), c, beta, delta, steps,
            g12_out, v, s);
        if (rc != SS_EUNSUPPORTED) return rc;
    }
    FusedCall a = {};
    a.model = model;
    a.n = n;
    a.p = p;
    a.eta = eta;
    a.e = e;
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    a.col = column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n);
    a.c = c;
    a.ccd = 1;
    a.penalty = penalty;
    a.lambda = lambda;
    a.beta = beta;
    a.delta = delta;
    a.steps = steps;
    a.want_log = g12_out != nullptr;
    a.obj_penalty = -1;
    // Fine-Gray with a 0/1 design: one launch per coordinate, each carrying
    // the weighted totals of the next column (a totals pass only before the
    // first one); valued designs: a totals pass before every scan
    const bool fg_carry = model == SS_FINE_GRAY && vals_sorted == nullptr;
    for (int64_t j = j_begin; j < j_end; ++j) {
        a.j = (int32_t)j;
        a.jprev = j > j_begin ? (int32_t)(j - 1) : -1;
        a.step_prev = j > j_begin ? steps + (j - 1) : nullptr;
        a.out = g12_out ? g12_out + 3 * j : v.hdr->scratch_out;
        a.fg_have_totals = fg_carry && j > j_begin;
        a.jnext = fg_carry && j + 1 < j_end ? (int32_t)(j + 1) : -1;
        int32_t rc = launch_fused(a, v, s);
        if (rc) return rc;
    }
    return launch_apply(n, (int32_t)(j_end - 1), steps + (j_end - 1), eta, e, a.col, s);
}

int32_t ss_exp(int64_t n, const double *eta, double *e, void *stream)
{
    if (n < 1 || n > INT32_MAX || !eta || !e) return SS_EINVAL;
    return launch_exp(n, eta, e, (hipStream_t)stream);
}

int32_t ss_gather(int64_t n, const int32_t *perm, const double *src, double *dst,
                  void *stream)
{
    if (n < 1 || n > INT32_MAX || !perm || !src || !dst) return SS_EINVAL;
    return launch_gather(n, perm, src, dst, (hipStream_t)stream);
}

int32_t ss_exp_f32(int64_t n, const double *eta, float *e32, double *shift, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (n < 1 || n > INT32_MAX || !eta || !e32 || !shift) return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    return launch_exp_f32(n, eta, e32, shift, v, (hipStream_t)stream);
}

int32_t ss_grad_hess_mixed(int32_t model, int32_t acc, int64_t n, int64_t p, int64_t j,
                           const float *e32, const uint8_t *d8, const int32_t *d32,
                           const double *w_comp, const double *g_end,
                           const int64_t *col_ptr, const int32_t *rows_sorted,
                           const double *vals_sorted, const int32_t *chunk_ptr,
                           const double *c, double *out, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (acc != SS_ACC_F32 && acc != SS_ACC_F32_COMP && acc != SS_ACC_F64 &&
        acc != SS_ACC_F32_C64)
        return SS_EINVAL;
    if (bad_size(n, p) || j < 0 || j >= p) return SS_EINVAL;
    if (!e32 || !d8 || !d32) return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!w_comp || !g_end)) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !out) return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    return launch_mixed(acc, model, n, p, (int32_t)j, e32, d8, d32, w_comp, g_end,
                        column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n), c, out, v,
                        (hipStream_t)stream);
}

int32_t ss_grad_hess_f32(int32_t model, int32_t acc, int64_t n, int64_t p, int64_t j,
                         const float *e32, const uint8_t *d8, const int32_t *d32,
                         const double *w_comp, const double *g_end, const int64_t *col_ptr,
                         const int32_t *rows_sorted, const double *vals_sorted,
                         const int32_t *chunk_ptr, const double *c, double *out, void *ws,
                         size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (acc != SS_ACC_F64 && acc != SS_ACC_F32_C64) return SS_EINVAL;
    if (bad_size(n, p) || j < 0 || j >= p) return SS_EINVAL;
    if (!e32 || !aligned(e32, 16) || !d8 || !aligned(d8, 8) || !d32) return SS_EINVAL;
    if (model == SS_FINE_GRAY &&
        (!w_comp || !g_end || !aligned(w_comp, 16) || !aligned(g_end, 16)))
        return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !out) return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    FusedCall a = {};
    a.model = model;
    a.n = n;
    a.p = p;
    a.j = (int32_t)j;
    a.jprev = -1;
    a.jnext = -1;
    a.e32 = e32;
    a.f32_sums = acc == SS_ACC_F32_C64;
    a.d8 = d8;
    a.d32 = d32;
    a.w_comp = w_comp;
    a.g_end = g_end;
    a.col = column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n);
    a.c = c;
    a.out = out;
    a.want_log = 1;
    a.obj_penalty = -1;
    return launch_fused(a, v, (hipStream_t)stream);
}

int32_t ss_autotune_grad_hess(int32_t model, int32_t storage, int64_t n, int64_t p, int64_t j,
                              const void *e, const uint8_t *d8, const int32_t *d32,
                              const double *w_comp, const double *g_end,
                              const int64_t *col_ptr, const int32_t *rows_sorted,
                              const double *vals_sorted, const int32_t *chunk_ptr,
                              const double *c, double *out, void *ws, size_t ws_bytes,
                              int32_t reps, int32_t *choice, float *us, void *stream)
{
    if (reps < 1 || reps > 1000 || !choice) return SS_EINVAL;
    if (storage != SS_STORAGE_F64 && storage != SS_STORAGE_F32 &&
        storage != SS_STORAGE_F32_SUMS32)
        return SS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    auto call = [&]() -> int32_t {
        if (storage == SS_STORAGE_F64)
            return ss_grad_hess(model, n, p, j, (const double *)e, d8, d32, w_comp, g_end,
                                col_ptr, rows_sorted, vals_sorted, chunk_ptr, c, out, ws,
                                ws_bytes, stream);
        return ss_grad_hess_f32(model, storage == SS_STORAGE_F32 ? SS_ACC_F64 : SS_ACC_F32_C64,
                                n, p, j, (const float *)e, d8, d32, w_comp, g_end, col_ptr,
                                rows_sorted, vals_sorted, chunk_ptr, c, out, ws, ws_bytes,
                                stream);
    };
    // the arguments are checked by a first call with the current choice
    int32_t rc = call();
    if (rc != SS_OK) return rc;
    EventPair ev;
    SS_HIP_CHECK(hipEventCreate(&ev.a));
    SS_HIP_CHECK(hipEventCreate(&ev.b));
    static const int32_t cands[4] = {4, 8, 16, 32};
    float t[4];
    int32_t best = 0;
    for (int i = 0; i < 4; ++i) {
        ForceScope force(SS_TUNE_GRAD_HESS, cands[i]);
        for (int w = 0; w < 2; ++w)
            if ((rc = call()) != SS_OK) return rc;
        SS_HIP_CHECK(hipEventRecord(ev.a, s));
        for (int r = 0; r < reps; ++r)
            if ((rc = call()) != SS_OK) return rc;
        SS_HIP_CHECK(hipEventRecord(ev.b, s));
        SS_HIP_CHECK(hipEventSynchronize(ev.b));
        float ms = 0.f;
        SS_HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b));
        t[i] = ms * 1000.f / (float)reps;
        if (!best || t[i] < t[best - 1]) best = i + 1;
    }
    *choice = cands[best - 1];
    if (us)
        for (int i = 0; i < 4; ++i) us[i] = t[i];
    return ss_tune_set(SS_TUNE_GRAD_HESS, model, storage, vals_sorted != nullptr, n, *choice);
}

int32_t ss_autotune_sweep(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                          int64_t j_begin, int64_t j_end, const double *eta, const double *e,
                          const uint8_t *d8, const int32_t *d32, const double *w_comp,
                          const double *g_end, const int64_t *col_ptr,
                          const int32_t *rows_sorted, const double *vals_sorted,
                          const int32_t *chunk_ptr, const double *c, const double *beta,
                          const double *delta, double *eta_s, double *e_s, double *beta_s,
                          double *delta_s, double *steps_s, void *ws, size_t ws_bytes,
                          int32_t reps, int32_t *choice, float *us, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && penalty != SS_PENALTY_L1 && penalty != SS_PENALTY_L2)
        return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && !(lambda > 0.0)) return SS_EINVAL;
    if (bad_size(n, p) || j_begin < 0 || j_end > p || j_begin >= j_end) return SS_EINVAL;
    if (reps < 1 || reps > 1000 || !choice) return SS_EINVAL;
    if (!model_arrays_ok(model, e, d8, d32, w_comp, g_end) || !eta) return SS_EINVAL;
    if (!model_arrays_ok(model, e_s, d8, d32, w_comp, g_end) || !eta_s) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr || !c || !beta || !delta || !beta_s ||
        !delta_s || !steps_s)
        return SS_EINVAL;
    WsView v;
    if (!fused_ws_view(ws, ws_bytes, n, &v)) return SS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const Column col = column(col_ptr, rows_sorted, vals_sorted, chunk_ptr, n);
    auto restore = [&]() -> int32_t {
        SS_HIP_CHECK(hipMemcpyAsync(eta_s, eta, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        SS_HIP_CHECK(hipMemcpyAsync(e_s, e, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        SS_HIP_CHECK(hipMemcpyAsync(beta_s, beta, p * sizeof(double), hipMemcpyDeviceToDevice, s));
        SS_HIP_CHECK(hipMemcpyAsync(delta_s, delta, p * sizeof(double), hipMemcpyDeviceToDevice,
                                    s));
        return SS_OK;
    };
    auto sweep = [&]() {
        return sweep_persistent(model, penalty, lambda, n, j_begin, j_end, eta_s, e_s, d8, d32,
                                w_comp, g_end, col, c, beta_s, delta_s, steps_s, nullptr, v, s);
    };
    EventPair ev;
    SS_HIP_CHECK(hipEventCreate(&ev.a));
    SS_HIP_CHECK(hipEventCreate(&ev.b));
    static const int32_t cands[4] = {25616, 51208, 25608, 51216};
    float t[4];
    int32_t best = 0;
    for (int i = 0; i < 4; ++i) {
        t[i] = -1.f;
        if (model == SS_FINE_GRAY && cands[i] == 51216) continue;
        ForceScope force(SS_TUNE_SWEEP, cands[i]);
        int32_t rc = restore();
        if (rc != SS_OK) return rc;
        rc = sweep();
        if (rc == SS_EUNSUPPORTED) continue;  // does not fit on the device
        if (rc != SS_OK) return rc;
        float total = 0.f;
        for (int r = 0; r < reps; ++r) {
            if ((rc = restore()) != SS_OK) return rc;
            SS_HIP_CHECK(hipEventRecord(ev.a, s));
            if ((rc = sweep()) != SS_OK) return rc;
            SS_HIP_CHECK(hipEventRecord(ev.b, s));
            SS_HIP_CHECK(hipEventSynchronize(ev.b));
            float ms = 0.f;
            SS_HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b));
            total += ms;
        }
        t[i] = total * 1000.f / (float)reps;
        if (!best || t[i] < t[best - 1]) best = i + 1;
    }
    if (us)
        for (int i = 0; i < 4; ++i) us[i] = t[i];
    if (!best) return SS_EUNSUPPORTED;
    *choice = cands[best - 1];
    return ss_tune_set(SS_TUNE_SWEEP, model, SS_STORAGE_F64, vals_sorted != nullptr, n,
                       *choice);
}

size_t ss_eta_gradient_workspace_bytes(int64_t n)
{
    if (n < 1 || n > INT32_MAX) return 0;
    return adjoint_ws_bytes(n);
}

int32_t ss_gather_u8(int64_t n, const int32_t *perm, const uint8_t *src, uint8_t *dst,
                     void *stream)
{
    if (n < 1 || n > INT32_MAX || !perm || !src || !dst) return SS_EINVAL;
    return launch_gather_u8(n, perm, src, dst, (hipStream_t)stream);
}

int32_t ss_eta_gradient(int32_t model, int64_t n, const int32_t *inv_perm,
                        const int8_t *status_sorted, const double *eta, const double *e,
                        const uint8_t *d8, const int32_t *d32, const double *w_comp,
                        const double *g_end, double *grad, double *loglik, void *ws,
                        size_t ws_bytes, void *stream)
{
    const int8_t *status = status_sorted;
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (n < 1 || n > INT32_MAX) return SS_EINVAL;
    if (!inv_perm || !status || !eta || !e || !d8 || !d32 || !grad || !loglik) return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!w_comp || !g_end)) return SS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < adjoint_ws_bytes(n)) return SS_EWORKSPACE;
    return launch_eta_gradient(model, n, inv_perm, status, eta, e, d8, d32, w_comp, g_end, grad,
                               loglik, ws, (hipStream_t)stream);
}

size_t ss_beta_gradient_workspace_bytes(int64_t n, int64_t p)
{
    if (bad_size(n, p)) return 0;
    return beta_ws_bytes(n, p);
}

int32_t ss_beta_gradient(int32_t model, int64_t n, int64_t p, const int32_t *inv_perm,
                         const int8_t *status_sorted, const double *eta, const double *e,
                         const uint8_t *d8, const int32_t *d32, const double *w_comp,
                         const double *g_end, const int64_t *col_ptr,
                         const int32_t *rows_sorted, const double *vals_sorted,
                         const int32_t *chunk_ptr, double *grad_beta, double *grad_eta,
                         double *loglik, void *ws, size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (bad_size(n, p)) return SS_EINVAL;
    if (!status_sorted || !eta || !e || !d8 || !d32 || !grad_beta || !loglik) return SS_EINVAL;
    if (!col_ptr || !rows_sorted || !chunk_ptr) return SS_EINVAL;
    if (grad_eta && !inv_perm) return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!w_comp || !g_end)) return SS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < beta_ws_bytes(n, p)) return SS_EWORKSPACE;
    return launch_beta_gradient(model, n, p, inv_perm, status_sorted, eta, e, d8, d32, w_comp,
                                g_end, col_ptr, rows_sorted, vals_sorted, chunk_ptr, grad_beta,
                                grad_eta, loglik, ws, (hipStream_t)stream);
}

int64_t ss_cv_stride(int64_t n)
{
    if (n < 1 || n > INT32_MAX) return 0;
    return cv_stride(n);
}

size_t ss_cv_prepare_workspace_bytes(int64_t n, int32_t reps)
{
    if (n < 1 || n > INT32_MAX || reps < 1 || reps > 65535) return 0;
    return (size_t)reps * (size_t)(cv_stride(n) / 8);
}

static bool bad_cv(int64_t n, int64_t p, int32_t reps)
{
    return bad_size(n, p) || reps < 1 || reps > 65535;
}

int32_t ss_cv_prepare(int32_t model, int64_t n, int64_t p, int32_t reps, const int32_t *perm,
                      const int8_t *status, const double *y, const uint8_t *d8,
                      const uint8_t *train, const int64_t *col_ptr, const int32_t *rows_sorted,
                      const double *vals_sorted, uint8_t *train_s, uint8_t *d8_r,
                      int32_t *d32_r, uint32_t *xbits, double *c_r, double *w_r, double *g_r,
                      double *g_h, void *ws, size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (vals_sorted) return SS_EUNSUPPORTED;
    if (bad_cv(n, p, reps)) return SS_EINVAL;
    if (!perm || !status || !d8 || !train || !col_ptr || !rows_sorted || !train_s || !d8_r ||
        !d32_r || !xbits || !c_r)
        return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!y || !w_r || !g_r || !g_h)) return SS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < ss_cv_prepare_workspace_bytes(n, reps))
        return SS_EWORKSPACE;
    return launch_cv_prepare(model, n, p, reps, perm, status, y, d8, train, col_ptr,
                             rows_sorted, train_s, d8_r, d32_r, xbits, c_r, w_r, g_r, g_h, ws,
                             (hipStream_t)stream);
}

int32_t ss_cv_exp(int64_t n, int32_t reps, const double *eta, const uint8_t *train_s,
                  double *e, void *stream)
{
    if (n < 1 || n > INT32_MAX || reps < 1 || reps > 65535) return SS_EINVAL;
    if (!eta || !train_s || !e) return SS_EINVAL;
    return launch_cv_exp(n, reps, eta, train_s, e, (hipStream_t)stream);
}

size_t ss_cv_workspace_bytes(int32_t reps)
{
    if (reps < 1 || reps > 65535) return 0;
    return cv_ws_bytes(reps);
}

int32_t ss_cv_sweep(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                    int32_t reps, int64_t j_begin, int64_t j_end, double *eta, double *e,
                    const uint8_t *d8_r, const int32_t *d32_r, const uint8_t *train_s,
                    const uint32_t *xbits, const double *c_r, const double *w_r,
                    const double *g_r, double *beta, double *delta, double *g12_out, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (model == SS_FINE_GRAY && (!w_r || !g_r)) return SS_EINVAL;
    if (penalty != SS_PENALTY_NONE && penalty != SS_PENALTY_L1 && penalty != SS_PENALTY_L2)
        return SS_EUNSUPPORTED;
    if (penalty != SS_PENALTY_NONE && !(lambda > 0.0)) return SS_EINVAL;
    if (bad_cv(n, p, reps) || j_begin < 0 || j_end < j_begin || j_end > p) return SS_EINVAL;
    if (!eta || !e || !d8_r || !d32_r || !train_s || !xbits || !c_r || !beta || !delta)
        return SS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < cv_ws_bytes(reps)) return SS_EWORKSPACE;
    return launch_cv_sweep(model, penalty, lambda, n, p, reps, j_begin, j_end, eta, e, d8_r,
                           d32_r, train_s, xbits, c_r, w_r, g_r, beta, delta, g12_out, ws,
                           (hipStream_t)stream);
}

int32_t ss_cv_loglik(int32_t model, int64_t n, int32_t reps, const int32_t *perm,
                     const int8_t *status, const double *eta, const double *e,
                     const uint8_t *train_s, const uint8_t *d8, const int32_t *d32,
                     const uint8_t *d8_r, const int32_t *d32_r, const double *w_r,
                     const double *g_r, const double *g_h, double *out, void *stream)
{
    if (model != SS_COX && model != SS_FINE_GRAY) return SS_EUNSUPPORTED;
    if (n < 1 || n > INT32_MAX || reps < 1 || reps > 65535) return SS_EINVAL;
    if (!perm || !status || !eta || !e || !train_s || !d8 || !d32 || !d8_r || !d32_r || !out)
        return SS_EINVAL;
    if (model == SS_FINE_GRAY && (!w_r || !g_r || !g_h)) return SS_EINVAL;
    return launch_cv_loglik(model, n, reps, perm, status, eta, e, train_s, d8, d32, d8_r,
                            d32_r, w_r, g_r, g_h, out, (hipStream_t)stream);
}

int32_t ss_cv_select(int32_t n_gamma, int32_t reps, const double *scores, double *mean,
                     int32_t *best, void *stream)
{
    if (n_gamma < 1 || reps < 1 || reps > 65535) return SS_EINVAL;
    if (!scores || !mean || !best) return SS_EINVAL;
    return launch_cv_select(n_gamma, reps, scores, mean, best, (hipStream_t)stream);
}

}  // extern "C"
