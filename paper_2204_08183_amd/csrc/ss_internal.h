// Internal declarations shared by the survscan HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "survscan.h"

namespace ss {

constexpr int kWave = 64;

// ------------------------------------------------------------ host helpers
// Records the last HIP error for ss_status_string and maps it to a status.
int32_t record_hip_error(hipError_t err);
#define SS_HIP_CHECK(call)                                   \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return ss::record_hip_error(_e); \
    } while (0)
#define SS_LAUNCH_CHECK() SS_HIP_CHECK(hipGetLastError())

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ device helpers
// Cross-workgroup exchange on gfx950.  The eight XCDs of an MI355X each have
// their own L2, and an agent-scope acquire or release fence writes back or
// invalidates a whole L2, which costs microseconds and serialises every
// workgroup of the XCD behind it.  So the values exchanged between
// workgroups (look-back states, partial sums, counters) are only ever
// written and read with agent-scope atomic stores and loads, which the
// hardware performs at the device coherence point, and the two fences below
// only order those accesses: all outstanding vector memory operations of the
// wave complete (s_waitcnt vmcnt(0)), and a workgroup-scope fence keeps the
// compiler from moving accesses across.
__device__ __forceinline__ void order_release()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0); expcnt, lgkmcnt unchanged
}
__device__ __forceinline__ void order_acquire()
{
    __builtin_amdgcn_s_waitcnt(0xF70);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint64_t ld_flag(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_relaxed(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed_u32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_u32(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_u64(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t fetch_add_relaxed(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// ------------------------------------------------------------ workspace
// Values that cross workgroups travel as 16-byte (value, tag) pairs, each
// written and read with one 16-byte agent-scope access (ss_device.h).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Layout of the workspace (every region 256-byte aligned), T = max_tiles,
// U = ceil(T / kGroup) + 1 tile groups and V = ceil(T / kLbGroup) + 1
// look-back groups:
//   WsHeader | lb[T][8] | glb[V][8] | part[T][8] | fg_part[T][4] | gpart[U][8] |
//   fg_gpart[U][4] | sw_agg[T][8] | sw_part[T][4] | sw_step[T] |
//   sw_pre[T][8] | sw_pub[kPubCopies][2][kMaxSweepBlocks][kPubSlotWords]
struct alignas(256) WsHeader {
    uint64_t epoch;       // number of completed fused launches
    uint64_t fg_epoch;    // number of completed Fine-Gray totals passes
    uint32_t error;       // sticky: a bounded wait gave up
    uint32_t pad;
    double fg_tot[3];     // Fine-Gray totals sum_r e_r x_r^m w_r, m = 0..2
    double scratch_out[4];
};

// Look-back pairs of a tile carry the tag (epoch << 2) | state with state
// 1 = tile aggregate, 2 = inclusive prefix (anything else: not published in
// this launch).  Partial-sum pairs carry (epoch << 1) | 1.
constexpr int kMaxComp = 6;
constexpr uint64_t kStateAgg = 1;
constexpr uint64_t kStateInc = 2;

// Tiles per group of the two-level reduction of the per-tile partial sums.
constexpr int kGroup = 64;

// Tiles per group of the two-level look-back (at most 64: a group's last
// tile sums its other members with one lane each).
#ifndef SS_LB_GROUP
#define SS_LB_GROUP 64
#endif
constexpr int kLbGroup = SS_LB_GROUP;
static_assert(kLbGroup >= 2 && kLbGroup <= 64, "look-back groups of 2 to 64 tiles");

// Upper bound on the number of workgroups (segments) of one persistent sweep.
constexpr int kMaxSweepBlocks = 512;

// Publications of the one-exchange persistent sweep: up to kPubCopies
// copies of every segment's publication, by round parity (16-byte words, at
// most kPubSlotWords of them), each copy in an area of its own; every
// workgroup reads one copy, so the all-to-all gather spreads over that
// many times as many memory lines.
#ifndef SS_PUB_COPIES
#define SS_PUB_COPIES 8
#endif
constexpr int kPubCopies = SS_PUB_COPIES;
constexpr int kPubSlotWords = 16;  // 256 bytes: ld_pairs2 reads two neighbouring slots
constexpr int64_t kSwPubWords = 2 * (int64_t)kPubCopies * kMaxSweepBlocks * kPubSlotWords;

// Upper bound on polls of one bounded wait before it gives up (each poll is
// an uncached load plus a short sleep, so this is on the order of a second).
constexpr uint32_t kSpinLimit = 1u << 20;

struct WsView {
    WsHeader *hdr;
    u32x4 *lb;        // [max_tiles][8]  look-back (aggregate / inclusive prefix)
    u32x4 *glb;       // [groups][8]     look-back of groups of 64 tiles
    u32x4 *part;      // [max_tiles][8]  per-tile partial sums
    u32x4 *fg_part;   // [max_tiles][4]  Fine-Gray totals pass, per tile
    u32x4 *gpart;     // [groups][8]     per-group partial sums
    u32x4 *fg_gpart;  // [groups][4]
    // persistent sweep
    u32x4 *sw_agg;    // [max_tiles][8]
    u32x4 *sw_part;   // [max_tiles][4]
    u32x4 *sw_step;   // [max_tiles]
    u32x4 *sw_pre;    // [max_tiles][8]
    u32x4 *sw_pub;    // [kPubCopies][2][kMaxSweepBlocks][kPubSlotWords]
    int64_t max_tiles;
};

#ifdef SS_TRACE_TIMES
// Phase timestamps of analysis builds live behind the regular workspace:
// 8 slots per tile (fused kernels) or 8 x 8 per workgroup (sweeps).
__device__ __forceinline__ uint64_t *trace_base(const WsView &ws)
{
    return reinterpret_cast<uint64_t *>(ws.sw_pub + kSwPubWords);
}
#endif

// Bytes of the workspace for problems of up to n positions (the layout
// above; tiles are at least SS_CHUNK positions).
constexpr size_t fused_ws_bytes(int64_t n)
{
    const int64_t tiles = ceil_div(n, SS_CHUNK) + 1;
    const int64_t groups = ceil_div(tiles, kGroup) + 1;
    const int64_t lb_groups = ceil_div(tiles, kLbGroup) + 1;
    size_t b = sizeof(WsHeader);
    b = align_up(b + 16 * 8 * (size_t)tiles, 256);   // lb
    b = align_up(b + 16 * 8 * (size_t)lb_groups, 256);  // glb
    b = align_up(b + 16 * 8 * (size_t)tiles, 256);   // part
    b = align_up(b + 16 * 4 * (size_t)tiles, 256);   // fg_part
    b = align_up(b + 16 * 8 * (size_t)groups, 256);  // gpart
    b = align_up(b + 16 * 4 * (size_t)groups, 256);  // fg_gpart
    b = align_up(b + 16 * 8 * (size_t)tiles, 256);   // sw_agg
    b = align_up(b + 16 * 4 * (size_t)tiles, 256);   // sw_part
    b = align_up(b + 16 * (size_t)tiles, 256);       // sw_step
    b = align_up(b + 16 * 8 * (size_t)tiles, 256);   // sw_pre
    b = align_up(b + 16 * (size_t)kSwPubWords, 256);   // sw_pub
#ifdef SS_TRACE_TIMES
    b = align_up(b + sizeof(uint64_t) * 64 * (size_t)tiles, 256);
#endif
    return b;
}
bool fused_ws_view(void *ws, size_t ws_bytes, int64_t n, WsView *v);

// ------------------------------------------------------------ argument checks
inline bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// The fused kernels read e, w_comp and g_end with 16-byte loads and d8 with
// 8-byte loads.
inline bool model_arrays_ok(int32_t model, const double *e, const uint8_t *d8,
                            const int32_t *d32, const double *w_comp,
                            const double *g_end)
{
    if (!e || !d8 || !d32) return false;
    if (!aligned(e, 16) || !aligned(d8, 8)) return false;
    if (model == SS_FINE_GRAY) {
        if (!w_comp || !g_end) return false;
        if (!aligned(w_comp, 16) || !aligned(g_end, 16)) return false;
    }
    return true;
}


// ------------------------------------------------------------ launchers
struct Column {
    const int64_t *col_ptr;
    const int32_t *rows;
    const double *vals;      // nullptr: 0/1 indicator design
    const int32_t *chunk_ptr;
    int64_t nchunk1;         // ss_chunk_count(n) + 1
};

struct FusedCall {
    int32_t model;
    int64_t n;
    int64_t p;
    int32_t j;               // column of g', g''; -1 for the likelihood only
    int32_t jprev;           // column whose pending step is applied; -1 none
    const double *step_prev; // device scalar: pending step of jprev
    double *eta;             // written only when jprev >= 0
    double *e;
    // FP32 storage of e (ss_grad_hess_f32): e32 replaces e; f32_sums selects
    // FP32 in-tile sums and transform with the FP64 carry between tiles
    const float *e32;
    int32_t f32_sums;
    const uint8_t *d8;
    const int32_t *d32;
    const double *w_comp;
    const double *g_end;
    Column col;
    const double *c;
    double *out;             // [3]
    // coordinate update in the last tile (a3)
    int32_t ccd;             // 0 no update, 1 update beta/delta/steps
    int32_t penalty;
    double lambda;
    double *beta;
    double *delta;
    double *steps;
    // likelihood mode: out[0] = beta' c - sum d log S0
    const double *beta_ll;
    int32_t want_log;
    // objective mode (with beta_ll): obj_penalty >= 0 writes out[0] = l + pi,
    // out[1] = l, out[2] = pi with pi the penalty of Sec. 2.3 at beta_ll
    int32_t obj_penalty;
    double obj_lambda;
    // Fine-Gray with a 0/1 design inside a sweep: the totals
    // sum e w x^m over column j are in hdr->fg_tot already (fg_have_totals,
    // carried by the previous launch), and jnext >= 0 asks the last tile to
    // carry the totals of column jnext over the e this coordinate's step
    // leaves behind
    int32_t fg_have_totals;
    int32_t jnext;
    // error reporting of calls without a caller-owned workspace: the first
    // tile of the call's first launch clears the error word, the last tile
    // of its last launch copies it to *err_out (0.0 or 1.0)
    int32_t clear_error;
    double *err_out;
};

int32_t launch_fused(const FusedCall &call, const WsView &ws,
                     hipStream_t stream);

// ------------------------------------------------------------ launch shapes
// Positions per thread of the single-pass fused kernel when nothing is
// tuned: tiles of 2048 positions up to 1.5 M positions, of 4096 above.
inline int32_t default_ipt(int64_t n) { return n <= ((int64_t)3 << 19) ? 8 : 16; }
// The tuned choice for a launch (0: none); see tune.hip.
int32_t tune_lookup(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n);
// A choice forced on the calling thread's launches of one kind while a
// tuning call times its candidates (choice 0: none).
struct TuneForce {
    int32_t kind;
    int32_t choice;
};
TuneForce &tune_force();

// The whole sweep j_begin..j_end-1 as one cooperative launch; returns
// SS_EUNSUPPORTED (launching nothing) when the problem does not fit on the
// device at once, and the caller then launches per coordinate.
struct SweepCall {
    int32_t model;
    int64_t n;
    int32_t j_begin;
    int32_t j_end;
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
};
int32_t launch_sweep_persistent(const SweepCall &call, const WsView &ws,
                                hipStream_t stream);
int32_t launch_apply(int64_t n, int32_t j, const double *step, double *eta,
                     double *e, const Column &col, hipStream_t stream);
int32_t launch_ccd_scalar(int32_t penalty, double lambda, int32_t j,
                          const double *g12, double *beta, double *delta,
                          double *step, hipStream_t stream);
// Deterministic FP64 add-scan of in[0..m) into out (may alias): forward or
// reverse (suffix), inclusive or exclusive; `sums` holds scan_sums_bytes(m).
int32_t scan_add_f64(const double *in, double *out, int64_t m, bool rev, bool excl,
                     void *sums, hipStream_t s);
size_t scan_sums_bytes(int64_t m);
// The first two passes of scan_add_f64 alone: sums[t] = the exclusive carry
// of scan tile t (tiles of 2048 items, in scan order), for a kernel that
// finishes the scan itself.
int32_t scan_carries_f64(const double *in, int64_t m, bool rev, void *sums, hipStream_t s);
size_t adjoint_ws_bytes(int64_t n);
size_t beta_ws_bytes(int64_t n, int64_t p);
int32_t launch_gather_u8(int64_t n, const int32_t *perm, const uint8_t *src, uint8_t *dst,
                         hipStream_t s);
int32_t launch_beta_gradient(int32_t model, int64_t n, int64_t p, const int32_t *inv_perm,
                             const int8_t *status_s, const double *eta, const double *e,
                             const uint8_t *d8, const int32_t *d32, const double *w_comp,
                             const double *g_end, const int64_t *col_ptr,
                             const int32_t *rows_sorted, const double *vals_sorted,
                             const int32_t *chunk_ptr, double *grad_beta, double *grad_eta,
                             double *loglik, void *ws, hipStream_t s);
int32_t launch_eta_gradient(int32_t model, int64_t n, const int32_t *inv_perm,
                            const int8_t *status_s,
                            const double *eta, const double *e, const uint8_t *d8,
                            const int32_t *d32, const double *w_comp, const double *g_end,
                            double *grad, double *loglik, void *ws, hipStream_t s);
int64_t cv_stride(int64_t n);
int32_t launch_cv_prepare(int32_t model, int64_t n, int64_t p, int32_t reps, const int32_t *perm,
                          const int8_t *status, const double *y, const uint8_t *d8,
                          const uint8_t *train, const int64_t *col_ptr,
                          const int32_t *rows_sorted, uint8_t *train_s, uint8_t *d8_r,
                          int32_t *d32_r, uint32_t *xbits, double *c_r, double *w_r,
                          double *g_r, double *g_h, void *ws, hipStream_t s);
int32_t launch_cv_exp(int64_t n, int32_t reps, const double *eta, const uint8_t *train_s,
                      double *e, hipStream_t s);
size_t cv_ws_bytes(int32_t reps);
int32_t launch_cv_sweep(int32_t model, int32_t penalty, double lambda, int64_t n, int64_t p,
                        int32_t reps, int64_t j_begin, int64_t j_end, double *eta, double *e,
                        const uint8_t *d8_r, const int32_t *d32_r, const uint8_t *train_s,
                        const uint32_t *xbits, const double *c_r, const double *w_r,
                        const double *g_r, double *beta, double *delta, double *g12_out,
                        void *ws, hipStream_t s);
int32_t launch_cv_loglik(int32_t model, int64_t n, int32_t reps, const int32_t *perm,
                         const int8_t *status, const double *eta, const double *e,
                         const uint8_t *train_s, const uint8_t *d8, const int32_t *d32,
                         const uint8_t *d8_r, const int32_t *d32_r, const double *w_r,
                         const double *g_r, const double *g_h, double *out, hipStream_t s);
int32_t launch_cv_select(int32_t n_gamma, int32_t reps, const double *scores, double *mean,
                         int32_t *best, hipStream_t s);
int32_t launch_mixed(int32_t acc, int32_t model, int64_t n, int64_t p, int32_t j,
                     const float *e32, const uint8_t *d8, const int32_t *d32,
                     const double *w_comp, const double *g_end, const Column &col,
                     const double *c, double *out, const WsView &ws, hipStream_t s);
int32_t launch_exp_f32(int64_t n, const double *eta, float *e32, double *shift,
                       const WsView &ws, hipStream_t s);
int32_t launch_exp(int64_t n, const double *eta, double *e,
                   hipStream_t stream);
int32_t launch_gather(int64_t n, const int32_t *perm, const double *src,
                      double *dst, hipStream_t stream);
int32_t launch_ws_init(void *ws, size_t bytes, hipStream_t stream);

// a0
size_t prepare_ws_bytes(int64_t n, int64_t p, int64_t nnz);
int32_t run_prepare(int32_t model, int64_t n, int64_t p, int64_t nnz,
                    const double *y, const int8_t *status,
                    const int64_t *col_ptr, const int32_t *rows,
                    const double *vals, int32_t *perm, int32_t *inv_perm,
                    uint8_t *d8, int32_t *d32, double *c,
                    int32_t *rows_sorted, double *vals_sorted,
                    int32_t *chunk_ptr, double *w_comp, double *g_end,
                    void *ws, size_t ws_bytes, hipStream_t stream);

// Device-side coordinate update shared by the fused epilogue and the
// standalone scalar kernel (Secs. 2.3-2.4).
__device__ __forceinline__ double ccd_newton_step(double g1, double g2,
                                                  double b, int penalty,
                                                  double lambda)
{
    if (penalty == SS_PENALTY_L2) {
        double d1 = g1 - b / lambda;
        double d2 = g2 - 1.0 / lambda;
        return d2 < 0.0 ? -d1 / d2 : 0.0;
    }
    if (!(g2 < 0.0)) return 0.0;
    if (penalty == SS_PENALTY_NONE) return -g1 / g2;
    // l1
    if (b != 0.0) {
        double s = b > 0.0 ? 1.0 : -1.0;
        double step = -(g1 - lambda * s) / g2;
        if ((b + step) * s < 0.0) step = -b;
        return step;
    }
    if (g1 - lambda > 0.0) return -(g1 - lambda) / g2;
    if (g1 + lambda < 0.0) return -(g1 + lambda) / g2;
    return 0.0;
}

__device__ __forceinline__ void ccd_apply(double g1, double g2, int penalty,
                                          double lambda, double *beta_j,
                                          double *delta_j, double *step_out)
{
    double b = *beta_j;
    double dj = *delta_j;
    double s = ccd_newton_step(g1, g2, b, penalty, lambda);
    double a = 0.0;
    if (s != 0.0) a = s > 0.0 ? fmin(s, dj) : -fmin(-s, dj);
    *beta_j = b + a;
    *delta_j = fmax(2.0 * fabs(s), 0.5 * dj);
    *step_out = a;
}

}  // namespace ss
