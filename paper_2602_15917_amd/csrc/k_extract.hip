// k_extract.hip - row spans, packed code stream with outliers, info structs.
//
// A row's span runs from its leftmost to its rightmost kept voxel.  Span
// lengths and "row has a span" flags are scanned together as one 64-bit
// value (flag << 40 | length), which gives every row its index in the row
// table and its first code.  The emit kernel then streams the span voxels
// once, recomputes their codes and stores them; outlier offsets come from a
// single-pass chained scan (decoupled look-back) over workgroups taken in
// ticket order, so the outlier array is filled in row order in the same pass.
#include "common.h"

namespace roix {

constexpr uint64_t kLenMask = (1ull << 40) - 1ull;
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62, kValMask = (1ull << 62) - 1ull;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ bool thread_exit_e(const DevState* S) {
    return __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

static int grid_rows(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------------------------ spans

__device__ __forceinline__ void put_span(const Layout& L, int64_t r, uint32_t xs, uint32_t xe, bool has) {
    L.row_xs[r] = xs;
    L.row_xe[r] = xe;
    L.row_packed[r] = has ? ((1ull << 40) | (uint64_t)(xe - xs)) : 0ull;
}

// from the runs: first and last run of a kept component
__global__ __launch_bounds__(kBlock) void k_spans_runs(Layout L, int64_t nrows) {
    const bool dead = thread_exit_e(L.S);
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += nthreads) {
        uint32_t xs = 0, xe = 0;
        bool has = false;
        if (!dead) {
            const uint32_t a0 = L.run_off[r], a1 = L.run_off[r + 1];
            for (uint32_t i = a0; i < a1; ++i) {
                if (!L.kept_flag[L.comp_id[L.parent[i]]]) continue;
                if (!has) xs = L.run_xs[i];
                xe = L.run_xe[i];
                has = true;
            }
        }
        put_span(L, r, xs, xe, has);
    }
}

hipError_t launch_spans_from_runs(const LaunchCtx& lc, const Geom& g, const Layout& L) {
    timer_begin(lc.timer, ST_SPANS, lc.stream);
    hipLaunchKernelGGL(k_spans_runs, dim3(grid_rows(g.nrows, kBlock, 16384)), dim3(kBlock), 0, lc.stream, L, g.nrows);
    timer_end(lc.timer, ST_SPANS, lc.stream);
    return hipGetLastError();
}

// from a per-voxel keep mask: one wave per row, ballots over 64 voxels
__global__ __launch_bounds__(kBlock) void k_spans_keep(Layout L, const uint8_t* __restrict__ keep, int64_t nx,
                                                       int64_t nrows) {
    const bool dead = thread_exit_e(L.S);
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = wave; r < nrows; r += nwaves) {
        uint32_t xs = 0xFFFFFFFFu, xe = 0;
        if (!dead) {
            const uint8_t* k = keep + r * nx;
            for (int64_t x0 = 0; x0 < nx; x0 += kWave) {
                const int64_t x = x0 + lane;
                const uint64_t m = __ballot(x < nx && k[x] != 0);
                if (m) {
                    if (xs == 0xFFFFFFFFu) xs = (uint32_t)(x0 + __ffsll((unsigned long long)m) - 1);
                    xe = (uint32_t)(x0 + 64 - __clzll((long long)m));
                }
            }
        }
        if (lane == 0) {
            const bool has = xs != 0xFFFFFFFFu;
            put_span(L, r, has ? xs : 0u, xe, has);
        }
    }
}

hipError_t launch_spans_from_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, const uint8_t* keep) {
    timer_begin(lc.timer, ST_SPANS, lc.stream);
    hipLaunchKernelGGL(k_spans_keep, dim3(grid_rows(g.nrows, kBlock / kWave, 16384)), dim3(kBlock), 0, lc.stream, L,
                       keep, g.nx, g.nrows);
    timer_end(lc.timer, ST_SPANS, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------------- emit

struct EmitOut {
    roix_row* rows;
    uint64_t rows_cap;
    uint8_t* stream;
    uint64_t stream_cap;  // bytes
    float* outl;
    uint64_t outl_cap;
};

// the code width is device data (it depends on the value range); the branch
// is uniform over the grid
__device__ __forceinline__ void store_code(uint8_t* stream, uint64_t idx, uint32_t u, int B) {
    if (B == 1)
        stream[idx] = (uint8_t)u;
    else if (B == 2)
        reinterpret_cast<uint16_t*>(stream)[idx] = (uint16_t)u;
    else
        reinterpret_cast<uint32_t*>(stream)[idx] = u;
}

// Workgroup = kEmitRows consecutive rows, taken in ticket order.  Phase 1:
// each wave streams its rows' spans, stores codes and counts outliers.  Then
// thread 0 publishes the workgroup's outlier count and looks back over the
// predecessors for its exclusive prefix.  Phase 2: row table entries and the
// outlier values (rows with outliers are read once more, from cache).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nrows,
                                                 Layout L, EmitOut o, int64_t n_blocks) {
    __shared__ uint32_t s_ticket;
    __shared__ int s_exit;
    __shared__ uint32_t s_cnt[kEmitRows];
    __shared__ unsigned long long s_excl;
    DevState* S = L.S;
    if (threadIdx.x == 0) {
        s_exit = thread_exit_e(S) ? 1 : 0;
        if (!s_exit) s_ticket = atomicAdd(&S->emit_ticket, 1u);
    }
    __syncthreads();
    if (s_exit) return;
    const int64_t blk = s_ticket;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    constexpr int kWaves = kBlock / kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    const uint32_t esc = S->esc;
    const int B = S->width_bits / 8;
    bool trunc = false;

    // phase 1: codes
    for (int lr = wave; lr < kEmitRows; lr += kWaves) {
        const int64_t row = blk * kEmitRows + lr;
        uint32_t cnt = 0;
        if (row < nrows) {
            const uint64_t packed = L.row_packed[row];  // exclusive scan value
            const uint32_t xs = L.row_xs[row], xe = L.row_xe[row];
            const uint64_t code0 = packed & kLenMask;
            // the span flag is only in the pre-scan value, so test the span itself
            if (xe > xs) {
                const T* src = in + (uint64_t)row * (uint64_t)nx + xs;
                const uint32_t len = xe - xs;
                for (uint32_t j0 = 0; j0 < len; j0 += kWave) {
                    const uint32_t j = j0 + lane;
                    bool isout = false;
                    if (j < len) {
                        const float x = (float)src[j];
                        const int32_t q = qcode(x, r);
                        isout = outlier(x, q, w, eb32);
                        const uint32_t u = isout ? esc : (uint32_t)(q - qmin);
                        const uint64_t idx = code0 + j;
                        if ((idx + 1) * (uint64_t)B <= o.stream_cap)
                            store_code(o.stream, idx, u, B);
                        else
                            trunc = true;
                    }
                    cnt += (uint32_t)__popcll(__ballot(isout));
                }
            }
        }
        if (lane == 0) s_cnt[lr] = cnt;
    }
    __syncthreads();

    // chained scan of outlier counts over workgroups
    if (threadIdx.x == 0) {
        unsigned long long agg = 0;
        for (int k = 0; k < kEmitRows; ++k) agg += s_cnt[k];
        uint64_t* lb = L.lookback;
        __hip_atomic_store(&lb[blk], kFlagAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long excl = 0;
        int64_t j = blk - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            const uint64_t v = __hip_atomic_load(&lb[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t f = v & ~kValMask;
            if (f == 0) {
                if (++spins > kSpinLimit) {
                    fail(S, ROIX_EDEVICE);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += v & kValMask;
            if (f == kFlagInc) break;
            --j;
        }
        __hip_atomic_store(&lb[blk], kFlagInc | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (blk == n_blocks - 1) S->n_outliers = excl + agg;
        s_excl = excl;
    }
    __syncthreads();

    // phase 2: row table and outlier values
    for (int lr = wave; lr < kEmitRows; lr += kWaves) {
        const int64_t row = blk * kEmitRows + lr;
        if (row >= nrows) continue;
        const uint32_t xs = L.row_xs[row], xe = L.row_xe[row];
        if (xe <= xs) continue;
        unsigned long long ooff = s_excl;
        for (int k = 0; k < lr; ++k) ooff += s_cnt[k];
        const uint64_t packed = L.row_packed[row];
        const uint64_t ridx = packed >> 40, code0 = packed & kLenMask;
        if (lane == 0) {
            if (ridx < o.rows_cap) {
                roix_row e;
                e.z = (uint32_t)(row / ny);
                e.y = (uint32_t)(row - (int64_t)e.z * ny);
                e.xs = xs;
                e.xe = xe;
                e.code_off = code0;
                e.outlier_off = ooff;
                o.rows[ridx] = e;
            } else {
                trunc = true;
            }
        }
        if (s_cnt[lr] == 0) continue;
        const T* src = in + (uint64_t)row * (uint64_t)nx + xs;
        const uint32_t len = xe - xs;
        unsigned long long k = ooff;
        for (uint32_t j0 = 0; j0 < len; j0 += kWave) {
            const uint32_t j = j0 + lane;
            bool isout = false;
            float x = 0.0f;
            if (j < len) {
                x = (float)src[j];
                isout = outlier(x, qcode(x, r), w, eb32);
            }
            const uint64_t m = __ballot(isout);
            if (isout) {
                const uint64_t below = m & ((1ull << lane) - 1ull);
                const unsigned long long at = k + (unsigned long long)__popcll(below);
                if (at < o.outl_cap)
                    o.outl[at] = x;
                else
                    trunc = true;
            }
            k += (unsigned long long)__popcll(m);
        }
    }
    if (trunc) atomicOr(&S->trunc, 1);
}

hipError_t launch_emit(const LaunchCtx& lc, const Geom& g, const Layout& L, const void* in, roix_dtype dt,
                       const roix_fused_out* out) {
    EmitOut o;
    o.rows = out->d_rows;
    o.rows_cap = out->d_rows ? (uint64_t)out->rows_cap : 0;
    o.stream = (uint8_t*)out->d_stream;
    o.stream_cap = out->d_stream ? (uint64_t)out->stream_cap_bytes : 0;
    o.outl = out->d_outliers;
    o.outl_cap = out->d_outliers ? (uint64_t)out->outliers_cap : 0;
    const int64_t nb = (g.nrows + kEmitRows - 1) / kEmitRows;
    timer_begin(lc.timer, ST_EMIT, lc.stream);
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_emit<float>, dim3((unsigned)nb), dim3(kBlock), 0, lc.stream, (const float*)in, g.nx,
                           g.ny, g.nrows, L, o, nb);
    else
        hipLaunchKernelGGL(k_emit<uint16_t>, dim3((unsigned)nb), dim3(kBlock), 0, lc.stream, (const uint16_t*)in,
                           g.nx, g.ny, g.nrows, L, o, nb);
    timer_end(lc.timer, ST_EMIT, lc.stream);
    return hipGetLastError();
}

// --------------------------------------------------------------- finalize

__global__ void k_finalize(const DevState* S, roix_quant_info* qi, roix_seg_info* si, roix_extract_info* ei,
                           int fused_q) {
    const int t = threadIdx.x;
    const int32_t st = S->status;
    if (qi && t == 0) {
        qi->status = S->qstatus;
        qi->xmin = S->xmin;
        qi->xmax = S->xmax;
        qi->eb32 = S->eb32;
        qi->w = S->w;
        qi->r = S->r;
        qi->qmin = S->qmin;
        qi->qmax = S->qmax;
        qi->K = S->K;
        qi->width_bits = S->width_bits;
        qi->esc = S->esc;
        qi->n_outliers = fused_q ? ROIX_NOT_COMPUTED : (S->qstatus ? 0ull : S->q_outliers);
    }
    if (si) {
        const bool qbad = S->qstatus != 0;
        si->hist[t] = qbad ? 0ull : S->hist[t];
        if (t == 0) {
            si->status = st;
            si->otsu_bin = qbad ? -1 : S->otsu_bin;
            si->q_thr = qbad ? 0 : S->q_thr;
            const bool seg_ok = st == 0;
            uint32_t flags = S->flags;
            if (seg_ok && S->n_kept == 0) flags |= ROIX_FLAG_EMPTY_ROI;
            si->flags = qbad ? 0u : flags;
            si->n_mask = qbad ? 0ull : S->n_mask;
            si->n_components = qbad ? 0ull : S->n_comps;
            si->n_kept = seg_ok ? S->n_kept : 0ull;
            si->n_kept_voxels = seg_ok ? S->n_kept_voxels : 0ull;
            const bool any = seg_ok && S->n_kept != 0;
            for (int k = 0; k < 6; ++k) si->bbox[k] = any ? S->bbox[k] : 0u;
        }
    }
    if (ei && t == 0) {
        const bool ok = st == 0;
        ei->status = st ? st : (S->trunc ? ROIX_ETRUNC : 0);
        ei->pad = 0;
        ei->n_rows = ok ? (S->span_total >> 40) : 0ull;
        ei->n_codes = ok ? (S->span_total & kLenMask) : 0ull;
        ei->n_outliers = ok ? S->n_outliers : 0ull;
        ei->stream_bytes = ok ? (S->span_total & kLenMask) * (uint64_t)(S->width_bits / 8) : 0ull;
    }
}

hipError_t launch_finalize(const LaunchCtx& lc, DevState* S, roix_quant_info* qi, roix_seg_info* si,
                           roix_extract_info* ei, bool fused_q) {
    timer_begin(lc.timer, ST_FINALIZE, lc.stream);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, lc.stream, (const DevState*)S, qi, si, ei, fused_q ? 1 : 0);
    timer_end(lc.timer, ST_FINALIZE, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
