// k_extract.hip - row spans, packed code stream with outliers, info structs.
//
// A row's span runs from its leftmost to its rightmost kept voxel.  Span
// lengths and "row has a span" flags are scanned together as one 64-bit
// value (flag << 40 | length), which gives every row its index in the row
// table and its first code.  The emit kernel then streams the span voxels
// once, recomputes their codes and stores them; outliers are stored in
// row order: the emit pass also counts each row's outliers, a scan turns the
// counts into offsets, and a second pass writes the row table and the
// outlier values (re-reading only rows that have outliers).
#include "common.h"

namespace roix {

constexpr uint64_t kLenMask = (1ull << 40) - 1ull;
constexpr int kEmitUnroll = 16;

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

template <int B>
struct CodeT;
template <>
struct CodeT<1> {
    using type = uint8_t;
};
template <>
struct CodeT<2> {
    using type = uint16_t;
};
template <>
struct CodeT<4> {
    using type = uint32_t;
};

// One wave per row: stream the span once (up to 64 * kEmitUnroll voxels in
// flight per wave), store the codes at the row's code offset and count the
// row's outliers.  B = bytes per code.
template <typename T, int B>
__device__ __forceinline__ void emit_codes_rows(const T* __restrict__ in, int64_t nx, int64_t nrows, const Layout& L,
                                                const EmitOut& o, bool& trunc) {
    using C = typename CodeT<B>::type;
    const DevState* S = L.S;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    const uint32_t esc = S->esc;
    C* codes = reinterpret_cast<C*>(o.stream);
    for (int64_t row = wave; row < nrows; row += nwaves) {
        const uint32_t xs = L.row_xs[row], xe = L.row_xe[row];
        uint32_t cnt = 0;
        if (xe > xs) {
            const uint64_t code0 = L.row_packed[row] & kLenMask;  // exclusive scan value
            const T* src = in + (uint64_t)row * (uint64_t)nx + xs;
            const uint32_t len = xe - xs;
            const bool fits = (code0 + len) * (uint64_t)B <= o.stream_cap;
            for (uint32_t j0 = 0; j0 < len; j0 += kWave * kEmitUnroll) {
                float xv[kEmitUnroll];
#pragma unroll
                for (int k = 0; k < kEmitUnroll; ++k) {
                    const uint32_t j = j0 + k * kWave + lane;
                    xv[k] = j < len ? (float)ld_stream(src + j) : 0.0f;
                }
#pragma unroll
                for (int k = 0; k < kEmitUnroll; ++k) {
                    const uint32_t j = j0 + k * kWave + lane;
                    const float x = xv[k];
                    const int32_t q = qcode(x, r);
                    const bool isout = j < len && outlier(x, q, w, eb32);
                    const uint32_t u = isout ? esc : (uint32_t)(q - qmin);
                    if (j < len) {
                        const uint64_t idx = code0 + j;
                        if (fits || (idx + 1) * (uint64_t)B <= o.stream_cap)
                            codes[idx] = (C)u;
                        else
                            trunc = true;
                    }
                    cnt += (uint32_t)__popcll(__ballot(isout));
                }
            }
        }
        if (lane == 0) L.row_outl[row] = cnt;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit_codes(const T* __restrict__ in, int64_t nx, int64_t nrows, Layout L,
                                                       EmitOut o) {
    DevState* S = L.S;
    if (thread_exit_e(S)) return;  // no barrier below
    bool trunc = false;
    const int B = S->width_bits / 8;  // uniform: one branch for the whole grid
    if (B == 1)
        emit_codes_rows<T, 1>(in, nx, nrows, L, o, trunc);
    else if (B == 2)
        emit_codes_rows<T, 2>(in, nx, nrows, L, o, trunc);
    else
        emit_codes_rows<T, 4>(in, nx, nrows, L, o, trunc);
    if (trunc) atomicOr(&S->trunc, 1);
}

// Pass 2 (after the scan of the outlier counts), one wave per row: the row
// table entry, and the outlier values of rows that have any (their spans are
// read once more).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit_rows(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nrows,
                                                      Layout L, EmitOut o) {
    DevState* S = L.S;
    if (thread_exit_e(S)) return;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const unsigned long long total = S->n_outliers;
    bool trunc = false;
    for (int64_t row = wave; row < nrows; row += nwaves) {
        const uint32_t xs = L.row_xs[row], xe = L.row_xe[row];
        if (xe <= xs) continue;
        const uint64_t packed = L.row_packed[row];
        const uint64_t ridx = packed >> 40, code0 = packed & kLenMask;
        const uint64_t ooff = L.row_outl[row];
        const uint64_t oend = row + 1 < nrows ? L.row_outl[row + 1] : total;
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
        if (oend == ooff) continue;
        const T* src = in + (uint64_t)row * (uint64_t)nx + xs;
        const uint32_t len = xe - xs;
        unsigned long long k = ooff;
        constexpr int U = 8;
        for (uint32_t j0 = 0; j0 < len; j0 += kWave * U) {
            float xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t j = j0 + u * kWave + lane;
                xv[u] = j < len ? (float)src[j] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t j = j0 + u * kWave + lane;
                const float x = xv[u];
                const bool isout = j < len && outlier(x, qcode(x, r), w, eb32);
                const uint64_t m = __ballot(isout);
                if (isout) {
                    const unsigned long long at = k + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
                    if (at < o.outl_cap)
                        o.outl[at] = x;
                    else
                        trunc = true;
                }
                k += (unsigned long long)__popcll(m);
            }
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
    const dim3 grid(grid_rows(g.nrows, kBlock / kWave, lc.grid_stream)), block(kBlock);
    timer_begin(lc.timer, ST_EMIT, lc.stream);
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_emit_codes<float>, grid, block, 0, lc.stream, (const float*)in, g.nx, g.nrows, L, o);
    else
        hipLaunchKernelGGL(k_emit_codes<uint16_t>, grid, block, 0, lc.stream, (const uint16_t*)in, g.nx, g.nrows, L, o);
    timer_end(lc.timer, ST_EMIT, lc.stream);
    hipError_t e = launch_scan_u64(lc, L.row_outl, L.row_outl, g.nrows, &L.S->n_outliers, L.scan_tmp);
    if (e != hipSuccess) return e;
    timer_begin(lc.timer, ST_EMIT_ROWS, lc.stream);
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_emit_rows<float>, grid, block, 0, lc.stream, (const float*)in, g.nx, g.ny, g.nrows, L, o);
    else
        hipLaunchKernelGGL(k_emit_rows<uint16_t>, grid, block, 0, lc.stream, (const uint16_t*)in, g.nx, g.ny, g.nrows,
                           L, o);
    timer_end(lc.timer, ST_EMIT_ROWS, lc.stream);
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
