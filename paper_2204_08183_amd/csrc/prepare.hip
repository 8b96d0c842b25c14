// One-time preparation of a data set on the GPU (gfx950):
//  - stable ordering by decreasing observed time (Sec. 2.7), by an LSD radix
//    sort whose in-tile ranks come from wave64 ballots, so equal times keep
//    increasing subject index;
//  - tie runs, events per run (Cox: status != 0, Fine-Gray: status == 1);
//  - Fine-Gray: Kaplan-Meier estimate of the censoring survival G (Sec. 2.2)
//    as a suffix product over runs, the competing-event weights 1/G(y) and
//    G(y) at every position;
//  - the CSC design re-labelled to sorted positions and sorted inside each
//    column, the per-column chunk index and c_j = sum over events of x_ij.
// Every integer output is produced with exact integer arithmetic, so it is
// identical from run to run.
#include <vector>

#include "scan_device.h"
#include "ss_internal.h"

namespace ss {

namespace {

// ------------------------------------------------------------ generic scan
// (block-level pieces in scan_device.h)

template <typename T, typename Op, bool REV>
__global__ __launch_bounds__(SB) void k_scan_reduce(const T *in, int64_t m, T *sums)
{
    __shared__ T s_w[SB / kWave];
    T it[SI];
    const int64_t base = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    load_items<T, Op, REV>(in, base, m, it);
    T tot = block_scan<T, Op>(it, Op::id(), s_w);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of sums[0..nb) in place.
template <typename T, typename Op>
__global__ __launch_bounds__(SB) void k_scan_spine(T *sums, int64_t nb)
{
    __shared__ T s_w[SB / kWave];
    __shared__ T s_last[SB / kWave];
    T carry = Op::id();
    for (int64_t c0 = 0; c0 < nb; c0 += ST) {
        T it[SI];
        const int64_t base = c0 + (int64_t)threadIdx.x * SI;
#pragma unroll
        for (int i = 0; i < SI; ++i) it[i] = base + i < nb ? sums[base + i] : Op::id();
        const T tot = block_scan<T, Op>(it, carry, s_w);
        inclusive_to_exclusive<T>(it, carry, s_last);
#pragma unroll
        for (int i = 0; i < SI; ++i)
            if (base + i < nb) sums[base + i] = it[i];
        carry = Op::op(carry, tot);
    }
}

template <typename T, typename Op, bool REV, bool EXCL>
__global__ __launch_bounds__(SB) void k_scan_down(const T *in, T *out, int64_t m,
                                                  const T *sums)
{
    __shared__ T s_w[SB / kWave];
    __shared__ T s_last[SB / kWave];
    T it[SI];
    const int64_t base = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    load_items<T, Op, REV>(in, base, m, it);
    const T carry = sums[blockIdx.x];
    block_scan<T, Op>(it, carry, s_w);
    if (EXCL) inclusive_to_exclusive<T>(it, carry, s_last);
    __syncthreads();  // `in` and `out` may alias: every read is done
    store_items<T, REV>(out, base, m, it);
}

// ------------------------------------------------------------ radix sort
constexpr int RB = 256;
constexpr int RI = 16;
constexpr int RT = RB * RI;

__global__ __launch_bounds__(RB) void k_radix_hist(const uint64_t *keys, int64_t m,
                                                   int shift, uint32_t *hist,
                                                   int64_t nb)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RT;
    for (int r = 0; r < RI; ++r) {
        const int64_t idx = base + (int64_t)r * RB + threadIdx.x;
        if (idx < m) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: items are visited in rounds of RB consecutive keys; inside
// a round a key's rank among equal digits comes from wave ballots (lanes in
// order) plus the counts of the earlier waves.
template <bool HAS_VAL>
__global__ __launch_bounds__(RB) void k_radix_scatter(const uint64_t *kin,
                                                      const uint64_t *vin, int64_t m,
                                                      int shift, const uint32_t *offs,
                                                      int64_t nb, uint64_t *kout,
                                                      uint64_t *vout, uint32_t *err)
{
    constexpr int NW = RB / kWave;
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wcnt[NW][256];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid / kWave;
    s_base[tid] = offs[(int64_t)tid * nb + blockIdx.x];
#pragma unroll
    for (int q = 0; q < NW; ++q) s_wcnt[q][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
    const int64_t base = (int64_t)blockIdx.x * RT;
    for (int r = 0; r < RI; ++r) {
        const int64_t idx = base + (int64_t)r * RB + tid;
        const bool valid = idx < m;
        const uint64_t key = valid ? kin[idx] : 0ull;
        const uint32_t digit = valid ? (uint32_t)((key >> shift) & 255u) : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t mb = __ballot(bit);
            peers &= bit ? mb : ~mb;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) s_wcnt[w][digit] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = s_base[digit] + rank;
            for (int q = 0; q < w; ++q) off += s_wcnt[q][digit];
            if ((int64_t)off < m) {
                kout[off] = key;
                if (HAS_VAL) vout[off] = vin[idx];
            } else {
                atomicOr(err, 32u);
            }
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            tot += s_wcnt[q][tid];
            s_wcnt[q][tid] = 0;
        }
        s_base[tid] += tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------ prepare steps
__device__ __forceinline__ uint64_t desc_key(double y)
{
    if (y == 0.0) y = 0.0;  // -0 and +0 are the same time
    uint64_t b = __double_as_longlong(y);
    const uint64_t asc = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    return ~asc;  // ascending key order = decreasing time
}

__global__ void k_time_keys(const double *y, int64_t n, uint64_t *keys, uint64_t *vals)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = desc_key(y[i]);
        vals[i] = (uint64_t)i;
    }
}

__global__ void k_after_sort(int64_t n, int model, const uint64_t *sorted_idx,
                             const double *y, const int8_t *status, int32_t *perm,
                             int32_t *inv_perm, double *y_s, int8_t *st_s,
                             uint8_t *ev_s, uint32_t *err)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = (int64_t)sorted_idx[k];
        if (i < 0 || i >= n) {
            atomicOr(err, 64u);
            i = 0;
        }
        perm[k] = (int32_t)i;
        inv_perm[i] = (int32_t)k;
        y_s[k] = y[i];
        int8_t s = status[i];
        if (s < 0 || s > 2) {
            atomicOr(err, 2u);
            s = 0;
        }
        st_s[k] = s;
        ev_s[k] = model == SS_COX ? (s != 0) : (s == 1);
    }
}

__global__ void k_run_start(int64_t n, const double *y_s, int32_t *start)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        start[k] = (k == 0 || y_s[k] != y_s[k - 1]) ? 1 : 0;
}

__global__ void k_fill_i32(int32_t *p, int64_t m, int32_t v)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// runid = inclusive scan of run starts, minus one
__global__ void k_run_counts(int64_t n, const int32_t *run_incl, const uint8_t *ev_s,
                             const int8_t *st_s, int32_t *cnt_ev, int32_t *cnt_cens,
                             uint32_t *err)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = run_incl[k] - 1;
        if (r < 0 || r >= n) {
            atomicOr(err, 128u);
            continue;
        }
        if (ev_s[k]) atomicAdd(&cnt_ev[r], 1);
        if (st_s[k] == 0) atomicAdd(&cnt_cens[r], 1);
    }
}

// d at run ends; Kaplan-Meier factor 1 - m_c / #{y >= c} at run ends
// (#{y >= c} = position of the run's last subject + 1).
__global__ void k_run_finish(int64_t n, const double *y_s, const int32_t *run_incl,
                             const int32_t *cnt_ev, const int32_t *cnt_cens,
                             uint8_t *d8, int32_t *d32, double *fac)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const bool end = (k == n - 1) || (y_s[k] != y_s[k + 1]);
        int32_t r = run_incl[k] - 1;
        if (r < 0 || r >= n) r = 0;  // reported by k_run_counts
        const int32_t d = end ? cnt_ev[r] : 0;
        d32[k] = d;
        d8[k] = (uint8_t)(d > 255 ? 255 : d);
        if (fac) {
            fac[k] = end ? 1.0 - (double)cnt_cens[r] / (double)(k + 1) : 1.0;
        }
    }
}

__global__ void k_fg_weights(int64_t n, const int8_t *st_s, const double *g_end,
                             double *w_comp)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        w_comp[k] = st_s[k] == 2 ? 1.0 / g_end[k] : 0.0;
}

// A balanced work list over the non-zeros: chunk q covers entries
// [begin, end) of column col, with at most kEntChunk entries.
constexpr int64_t kEntChunk = 4096;
struct EntChunk {
    int64_t col;
    int64_t begin;
    int64_t end;
};

__global__ void k_csc_keys(const EntChunk *chunks, int64_t nchunks, int64_t n,
                           const int32_t *rows, const double *vals,
                           const int32_t *inv_perm, int posbits, uint64_t *keys,
                           uint64_t *kv, uint32_t *err)
{
    for (int64_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
        const EntChunk ch = chunks[q];
        for (int64_t o = ch.begin + threadIdx.x; o < ch.end; o += blockDim.x) {
            int32_t r = rows[o];
            if (r < 0 || r >= n) {
                atomicOr(err, 8u);
                r = 0;
            }
            keys[o] = ((uint64_t)ch.col << posbits) | (uint64_t)inv_perm[r];
            if (vals) kv[o] = (uint64_t)__double_as_longlong(vals[o]);
        }
    }
}

__global__ void k_csc_unpack(int64_t nnz, const uint64_t *keys, const uint64_t *kv,
                             uint64_t posmask, int32_t *rows_sorted, double *vals_sorted)
{
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nnz;
         o += (int64_t)gridDim.x * blockDim.x) {
        rows_sorted[o] = (int32_t)(keys[o] & posmask);
        if (vals_sorted) vals_sorted[o] = __longlong_as_double((long long)kv[o]);
    }
}

// c_j, step 1: every chunk sums x over its event rows in a fixed order.
__global__ __launch_bounds__(256) void k_col_c_part(const EntChunk *chunks, int64_t nchunks,
                                                    int64_t n, const int32_t *rows_sorted,
                                                    const double *vals_sorted,
                                                    const uint8_t *ev_s, double *part)
{
    __shared__ double s_red[256 / kWave];
    for (int64_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
        const EntChunk ch = chunks[q];
        double acc = 0.0;
        for (int64_t o = ch.begin + threadIdx.x; o < ch.end; o += blockDim.x) {
            const int32_t r = rows_sorted[o];
            if (r >= 0 && r < n && ev_s[r]) acc += vals_sorted ? vals_sorted[o] : 1.0;
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane_id() == 0) s_red[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < 256 / kWave; ++i) t += s_red[i];
            part[q] = t;
        }
        __syncthreads();
    }
}

// c_j, step 2: one thread per column adds its chunks in order.
__global__ void k_col_c_final(int64_t p, const int64_t *col_first_chunk, const double *part,
                              double *c)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < p;
         j += (int64_t)gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int64_t q = col_first_chunk[j]; q < col_first_chunk[j + 1]; ++q) t += part[q];
        c[j] = t;
    }
}

// chunk_ptr[j*(C+1)+t] = first offset in column j with position >= t*SS_CHUNK.
// Step 1: every non-zero writes the boundaries between its predecessor's
// chunk and its own.
__global__ void k_chunk_ptr_entries(const EntChunk *chunks, int64_t nchunks, int64_t nchunk,
                                    const int64_t *col_ptr, const int32_t *rows_sorted,
                                    int32_t *chunk_ptr, uint32_t *err)
{
    for (int64_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
        const EntChunk ch = chunks[q];
        const int64_t c0 = col_ptr[ch.col];
        int32_t *cp = chunk_ptr + ch.col * (nchunk + 1);
        for (int64_t o = ch.begin + threadIdx.x; o < ch.end; o += blockDim.x) {
            const int32_t r = rows_sorted[o];
            int64_t cur = r / SS_CHUNK;
            if (r < 0 || cur >= nchunk) {
                atomicOr(err, 256u);
                continue;
            }
            int64_t prev = -1;
            if (o > c0) {
                const int32_t rp = rows_sorted[o - 1];
                if (rp >= r) atomicOr(err, 16u);  // duplicate row in a column
                prev = rp / SS_CHUNK;
                if (rp < 0 || prev > cur) prev = cur;
            }
            for (int64_t t = prev + 1; t <= cur; ++t) cp[t] = (int32_t)(o - c0);
        }
    }
}

// Step 2: the boundaries after the last non-zero of every column.
__global__ void k_chunk_ptr_tail(int64_t p, int64_t nchunk, const int64_t *col_ptr,
                                 const int32_t *rows_sorted, int32_t *chunk_ptr)
{
    for (int64_t j = blockIdx.x; j < p; j += gridDim.x) {
        const int64_t c0 = col_ptr[j];
        const int64_t m = col_ptr[j + 1] - c0;
        int64_t last = m == 0 ? -1 : rows_sorted[c0 + m - 1] / SS_CHUNK;
        if (last < -1 || last >= nchunk) last = nchunk - 1;
        int32_t *cp = chunk_ptr + j * (nchunk + 1);
        for (int64_t t = last + 1 + threadIdx.x; t <= nchunk; t += blockDim.x)
            cp[t] = (int32_t)m;
    }
}

int grid_1d(int64_t work, int cap = 8192)
{
    int64_t g = ceil_div(work, 256);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

int bits_for(int64_t v)  // bits needed for values in [0, v]
{
    int b = 0;
    while (b < 63 && (v >> b) != 0) ++b;
    return b;
}

// ------------------------------------------------------------ workspace
struct PrepWs {
    uint64_t *keyA, *keyB, *valA, *valB;
    uint32_t *hist;
    uint64_t *sums;       // scan spine (8-byte slots for any T)
    double *y_s;
    double *fac;
    int32_t *run_incl;
    int32_t *cnt_ev;
    int32_t *cnt_cens;
    int8_t *st_s;
    uint8_t *ev_s;
    uint32_t *err;
    EntChunk *chunks;
    double *part;
    int64_t *col_first;
};

size_t layout(int64_t n, int64_t p, int64_t nnz, char *base, PrepWs *w)
{
    const int64_t max_chunks = nnz / kEntChunk + p + 1;
    const int64_t m = n > nnz ? n : nnz;
    const int64_t nbr = ceil_div(m, RT);
    const int64_t hist_len = 256 * nbr;
    const int64_t scan_len = hist_len > n ? hist_len : n;
    const int64_t nbs = ceil_div(scan_len, ST) + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes, 256);
        return p;
    };
    PrepWs t;
    t.keyA = (uint64_t *)take(8 * (size_t)m);
    t.keyB = (uint64_t *)take(8 * (size_t)m);
    t.valA = (uint64_t *)take(8 * (size_t)m);
    t.valB = (uint64_t *)take(8 * (size_t)m);
    t.hist = (uint32_t *)take(4 * (size_t)hist_len);
    t.sums = (uint64_t *)take(8 * (size_t)nbs);
    t.y_s = (double *)take(8 * (size_t)n);
    t.fac = (double *)take(8 * (size_t)n);
    t.run_incl = (int32_t *)take(4 * (size_t)n);
    t.cnt_ev = (int32_t *)take(4 * (size_t)n);
    t.cnt_cens = (int32_t *)take(4 * (size_t)n);
    t.st_s = (int8_t *)take((size_t)n);
    t.ev_s = (uint8_t *)take((size_t)n);
    t.err = (uint32_t *)take(256);
    t.chunks = (EntChunk *)take(sizeof(EntChunk) * (size_t)max_chunks);
    t.part = (double *)take(8 * (size_t)max_chunks);
    t.col_first = (int64_t *)take(8 * (size_t)(p + 1));
    if (w) *w = t;
    return off;
}

template <typename T, typename Op, bool REV, bool EXCL>
int32_t device_scan(const T *in, T *out, int64_t m, uint64_t *sums_raw, hipStream_t s)
{
    if (m <= 0) return SS_OK;
    T *sums = (T *)sums_raw;
    const int64_t nb = ceil_div(m, ST);
    hipLaunchKernelGGL((k_scan_reduce<T, Op, REV>), dim3((unsigned)nb), dim3(SB), 0, s, in, m, sums);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_scan_spine<T, Op>), dim3(1), dim3(SB), 0, s, sums, nb);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_scan_down<T, Op, REV, EXCL>), dim3((unsigned)nb), dim3(SB), 0, s, in, out, m,
                       (const T *)sums);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

// Sorts (keyA, valA) by key bits [0, nbits); result in the returned buffers.
int32_t radix_sort(int64_t m, int nbits, bool has_val, PrepWs &w, uint64_t **keys_out,
                   uint64_t **vals_out, hipStream_t s)
{
    uint64_t *ka = w.keyA, *kb = w.keyB, *va = w.valA, *vb = w.valB;
    const int64_t nb = ceil_div(m, RT);
    for (int shift = 0; shift < nbits; shift += 8) {
        if (m > 0) {
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(RB), 0, s, ka, m, shift,
                               w.hist, nb);
            SS_LAUNCH_CHECK();
            int32_t rc = device_scan<uint32_t, OpAdd<uint32_t>, false, true>(
                w.hist, w.hist, 256 * nb, w.sums, s);
            if (rc) return rc;
            if (has_val)
                hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nb), dim3(RB), 0, s, ka,
                                   va, m, shift, w.hist, nb, kb, vb, w.err);
            else
                hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nb), dim3(RB), 0, s, ka,
                                   va, m, shift, w.hist, nb, kb, vb, w.err);
            SS_LAUNCH_CHECK();
        }
        uint64_t *t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    *keys_out = ka;
    *vals_out = va;
    return SS_OK;
}

}  // namespace

size_t prepare_ws_bytes(int64_t n, int64_t p, int64_t nnz)
{
    return layout(n, p, nnz, nullptr, nullptr);
}

int32_t run_prepare(int32_t model, int64_t n, int64_t p, int64_t nnz, const double *y,
                    const int8_t *status, const int64_t *col_ptr, const int32_t *rows,
                    const double *vals, int32_t *perm, int32_t *inv_perm, uint8_t *d8,
                    int32_t *d32, double *c, int32_t *rows_sorted, double *vals_sorted,
                    int32_t *chunk_ptr, double *w_comp, double *g_end, void *ws,
                    size_t ws_bytes, hipStream_t s)
{
    PrepWs w;
    if (layout(n, p, nnz, (char *)ws, &w) > ws_bytes) return SS_EWORKSPACE;
    const bool fg = model == SS_FINE_GRAY;
    int32_t rc;

    // ---- the column pointers on the host: checked there, and cut into a
    // balanced list of non-zero chunks for the design kernels
    std::vector<int64_t> cp_host((size_t)p + 1);
    SS_HIP_CHECK(hipMemcpyAsync(cp_host.data(), col_ptr, sizeof(int64_t) * (size_t)(p + 1),
                                hipMemcpyDeviceToHost, s));
    SS_HIP_CHECK(hipStreamSynchronize(s));
    if (cp_host[0] != 0 || cp_host[(size_t)p] != nnz) return SS_EINVAL;
    std::vector<EntChunk> chunks;
    std::vector<int64_t> first((size_t)p + 1);
    chunks.reserve((size_t)(nnz / kEntChunk + p + 1));
    for (int64_t j = 0; j < p; ++j) {
        const int64_t a = cp_host[(size_t)j], b = cp_host[(size_t)j + 1];
        if (b < a || a < 0 || b > nnz) return SS_EINVAL;
        first[(size_t)j] = (int64_t)chunks.size();
        for (int64_t o = a; o < b; o += kEntChunk)
            chunks.push_back(EntChunk{j, o, o + kEntChunk < b ? o + kEntChunk : b});
    }
    first[(size_t)p] = (int64_t)chunks.size();
    const int64_t nchunks = (int64_t)chunks.size();
    if (nchunks > 0)
        SS_HIP_CHECK(hipMemcpyAsync(w.chunks, chunks.data(), sizeof(EntChunk) * chunks.size(),
                                    hipMemcpyHostToDevice, s));
    SS_HIP_CHECK(hipMemcpyAsync(w.col_first, first.data(), sizeof(int64_t) * first.size(),
                                hipMemcpyHostToDevice, s));

    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)w.err, (int64_t)1, 0);
    SS_LAUNCH_CHECK();

    // ---- ordering by decreasing time, stable in the subject index
    hipLaunchKernelGGL(k_time_keys, dim3(grid_1d(n)), dim3(256), 0, s, y, n, w.keyA, w.valA);
    SS_LAUNCH_CHECK();
    uint64_t *ks, *vs;
    rc = radix_sort(n, 64, true, w, &ks, &vs, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_after_sort, dim3(grid_1d(n)), dim3(256), 0, s, n, (int)model, vs, y,
                       status, perm, inv_perm, w.y_s, w.st_s, w.ev_s, w.err);
    SS_LAUNCH_CHECK();

    // ---- tie runs and event counts
    hipLaunchKernelGGL(k_run_start, dim3(grid_1d(n)), dim3(256), 0, s, n, w.y_s, w.run_incl);
    SS_LAUNCH_CHECK();
    rc = device_scan<int32_t, OpAdd<int32_t>, false, false>(w.run_incl, w.run_incl, n, w.sums, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_1d(n)), dim3(256), 0, s, w.cnt_ev, n, 0);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_1d(n)), dim3(256), 0, s, w.cnt_cens, n, 0);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_run_counts, dim3(grid_1d(n)), dim3(256), 0, s, n, w.run_incl, w.ev_s,
                       w.st_s, w.cnt_ev, w.cnt_cens, w.err);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_run_finish, dim3(grid_1d(n)), dim3(256), 0, s, n, w.y_s, w.run_incl,
                       w.cnt_ev, w.cnt_cens, d8, d32, fg ? w.fac : (double *)nullptr);
    SS_LAUNCH_CHECK();

    // ---- Fine-Gray: Kaplan-Meier G as an inclusive suffix product
    if (fg) {
        rc = device_scan<double, OpMul<double>, true, false>(w.fac, g_end, n, w.sums, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_fg_weights, dim3(grid_1d(n)), dim3(256), 0, s, n, w.st_s, g_end,
                           w_comp);
        SS_LAUNCH_CHECK();
    }

    // ---- design: re-label to sorted positions, sort inside columns
    const int posbits = bits_for(n - 1);
    const int colbits = bits_for(p - 1);
    const unsigned gch = (unsigned)(nchunks < 65536 ? (nchunks > 0 ? nchunks : 1) : 65536);
    if (nnz > 0) {
        hipLaunchKernelGGL(k_csc_keys, dim3(gch), dim3(256), 0, s, w.chunks, nchunks, n, rows,
                           vals, inv_perm, posbits, w.keyA, w.valA, w.err);
        SS_LAUNCH_CHECK();
        rc = radix_sort(nnz, posbits + colbits, vals != nullptr, w, &ks, &vs, s);
        if (rc) return rc;
        const uint64_t posmask = posbits >= 64 ? ~0ull : ((1ull << posbits) - 1);
        hipLaunchKernelGGL(k_csc_unpack, dim3(grid_1d(nnz)), dim3(256), 0, s, nnz, ks, vs,
                           posmask, rows_sorted, vals ? vals_sorted : (double *)nullptr);
        SS_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_col_c_part, dim3(gch), dim3(256), 0, s, w.chunks, nchunks, n,
                           rows_sorted, vals ? vals_sorted : (const double *)nullptr, w.ev_s,
                           w.part);
        SS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_col_c_final, dim3(grid_1d(p)), dim3(256), 0, s, p, w.col_first,
                       w.part, c);
    SS_LAUNCH_CHECK();
    const int64_t nchunk = ceil_div(n, SS_CHUNK);
    if (nnz > 0) {
        hipLaunchKernelGGL(k_chunk_ptr_entries, dim3(gch), dim3(256), 0, s, w.chunks, nchunks,
                           nchunk, col_ptr, rows_sorted, chunk_ptr, w.err);
        SS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_chunk_ptr_tail, dim3((unsigned)(p < 8192 ? p : 8192)), dim3(256), 0, s,
                       p, nchunk, col_ptr, rows_sorted, chunk_ptr);
    SS_LAUNCH_CHECK();

    // ---- data errors found on the device
    uint32_t err = 0;
    SS_HIP_CHECK(hipMemcpyAsync(&err, w.err, sizeof(err), hipMemcpyDeviceToHost, s));
    SS_HIP_CHECK(hipStreamSynchronize(s));
    return err ? SS_EINVAL : SS_OK;
}

int32_t scan_add_f64(const double *in, double *out, int64_t m, bool rev, bool excl,
                     void *sums, hipStream_t s)
{
    uint64_t *w = reinterpret_cast<uint64_t *>(sums);
    if (rev) {
        return excl ? device_scan<double, OpAdd<double>, true, true>(in, out, m, w, s)
                    : device_scan<double, OpAdd<double>, true, false>(in, out, m, w, s);
    }
    return excl ? device_scan<double, OpAdd<double>, false, true>(in, out, m, w, s)
                : device_scan<double, OpAdd<double>, false, false>(in, out, m, w, s);
}

size_t scan_sums_bytes(int64_t m) { return 8 * (size_t)ceil_div(m, ST); }

int32_t scan_carries_f64(const double *in, int64_t m, bool rev, void *sums, hipStream_t s)
{
    if (m <= 0) return SS_OK;
    double *w = reinterpret_cast<double *>(sums);
    const int64_t nb = ceil_div(m, ST);
    if (rev)
        hipLaunchKernelGGL((k_scan_reduce<double, OpAdd<double>, true>), dim3((unsigned)nb),
                           dim3(SB), 0, s, in, m, w);
    else
        hipLaunchKernelGGL((k_scan_reduce<double, OpAdd<double>, false>), dim3((unsigned)nb),
                           dim3(SB), 0, s, in, m, w);
    SS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_scan_spine<double, OpAdd<double>>), dim3(1), dim3(SB), 0, s, w, nb);
    SS_LAUNCH_CHECK();
    return SS_OK;
}

}  // namespace ss
