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

// from the runs: first and last run of a kept component.  With one kept
// component of known root run, a run is kept when its root (parent, after
// the flattening) is that run: no lookup of the component's flag.
__device__ __forceinline__ void k_spans_runs_body(const VPart vp, Layout L, int64_t nrows) {
    const bool dead = thread_exit_e(L.S);
    const bool by_root = L.S->kept_by_root != 0;
    const uint32_t kr = L.S->kept_root;
    const int64_t nthreads = (int64_t)vp.n * blockDim.x;
    for (int64_t r = (int64_t)vp.b * blockDim.x + threadIdx.x; r < nrows; r += nthreads) {
        uint32_t xs = 0, xe = 0;
        bool has = false;
        if (!dead) {
            const uint32_t a0 = L.run_off[r], a1 = L.run_off[r + 1];
            for (uint32_t i = a0; i < a1; ++i) {
                const uint32_t root = L.parent[i];
                if (by_root ? root != kr : !L.kept_flag[L.comp_id[root]]) continue;
                if (!has) xs = L.run_xs[i];
                xe = L.run_xe[i];
                has = true;
            }
        }
        put_span(L, r, xs, xe, has);
    }
}
__global__ __launch_bounds__(kBlock) void k_spans_runs(Layout L, int64_t nrows) {
    k_spans_runs_body(hw_part(), L, nrows);
}

hipError_t launch_spans_from_runs(const LaunchCtx& lc, const Geom& g, const Layout& L) {
    timer_begin(lc.timer, ST_SPANS, lc.stream);
    launch_k<kBlock, k_spans_runs_body>(lc, k_spans_runs, dim3(grid_rows(g.nrows, kBlock, 16384)), dim3(kBlock), 0, L, g.nrows);
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
    uint64_t nvox;  // voxels of the input (bound of the whole-quad loads)
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

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Index of the flat code space, one thread per row: nz_rows[ridx] = row of
// the ridx-th span, span_desc[ridx] = its first code and voxel offset,
// chunk_row[q] = ridx of the span holding code q * chunk.  Also clears the
// per-row outlier counters.
__device__ __forceinline__ void k_emit_index_body(const VPart vp, Layout L, int64_t nx, int64_t nrows) {
    if (thread_exit_e(L.S)) return;
    if (vp.b == 0 && threadIdx.x == 0) L.S->n_slow = 0u;
    const int64_t nthreads = (int64_t)vp.n * blockDim.x;
    for (int64_t r = (int64_t)vp.b * blockDim.x + threadIdx.x; r < nrows; r += nthreads) {
        L.row_outl[r] = 0ull;
        const uint32_t xs = L.row_xs[r], xe = L.row_xe[r];
        if (xe <= xs) continue;
        const uint64_t packed = L.row_packed[r];
        const uint32_t ridx = (uint32_t)(packed >> 40);
        const uint64_t code0 = packed & kLenMask, code1 = code0 + (xe - xs);
        L.nz_rows[ridx] = (uint32_t)r;
        // descriptor for the emit: first code, and voxel = code + offset
        const uint64_t off = row_origin(L, (uint32_t)r, nx) + xs - code0;
        *reinterpret_cast<uint4*>(L.span_desc + 2 * (uint64_t)ridx) =
            make_uint4((uint32_t)code0, (uint32_t)(code0 >> 32), (uint32_t)off, (uint32_t)(off >> 32));
        for (uint64_t q = (code0 + kEmitChunk - 1) / kEmitChunk; q * kEmitChunk < code1; ++q) L.chunk_row[q] = ridx;
    }
}
__global__ __launch_bounds__(kBlock) void k_emit_index(Layout L, int64_t nx, int64_t nrows) {
    k_emit_index_body(hw_part(), L, nx, nrows);
}

// Four consecutive input values starting at voxel v.  float: one 16-byte
// load (the ISA needs only 4-byte alignment for multi-dword loads).  uint16:
// one 12-byte load from the 4-byte-aligned voxel at or before v.
__device__ __forceinline__ void load_quad(const float* in, uint64_t v, float (&x)[4]) {
    const v4u32_t q = __builtin_nontemporal_load(reinterpret_cast<const v4u32_t*>(in + v));
    x[0] = __uint_as_float(q.x);
    x[1] = __uint_as_float(q.y);
    x[2] = __uint_as_float(q.z);
    x[3] = __uint_as_float(q.w);
}
// Elements a whole-quad load at voxel v reads, counted from v: a quad is
// loaded whole only when v + quad_reach <= the voxel count.
template <typename T>
__device__ __forceinline__ constexpr uint64_t quad_reach() {
    return sizeof(T) == 4 ? 4 : 6;
}
__device__ __forceinline__ void load_quad(const uint16_t* in, uint64_t v, float (&x)[4]) {
    const uint64_t v0 = v & ~1ull;
    const v3u32_t q = *(reinterpret_cast<const v3u32_t*>(in + v0));
    const uint32_t sh = (uint32_t)(v - v0) * 16u;
    const uint64_t lo = ((uint64_t)q.y << 32) | q.x, hi = ((uint64_t)q.z << 32) | q.y;
    const uint64_t a = sh ? (lo >> 16) | ((uint64_t)q.z << 48) : lo;  // values v .. v+3
    (void)hi;
    x[0] = (float)(uint32_t)(a & 0xFFFFu);
    x[1] = (float)(uint32_t)((a >> 16) & 0xFFFFu);
    x[2] = (float)(uint32_t)((a >> 32) & 0xFFFFu);
    x[3] = (float)(uint32_t)(a >> 48);
}

template <int B>
__device__ __forceinline__ void store_quad(uint8_t* stream, uint64_t c, const uint32_t (&u)[4]) {
    if constexpr (B == 1) {
        *reinterpret_cast<uint32_t*>(stream + c) = u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24);
    } else if constexpr (B == 2) {
        *reinterpret_cast<uint2*>(stream + 2 * c) = make_uint2(u[0] | (u[1] << 16), u[2] | (u[3] << 16));
    } else {
        *reinterpret_cast<uint4*>(stream + 4 * c) = make_uint4(u[0], u[1], u[2], u[3]);
    }
}

// Codes of one chunk [c0, c1) whose spans are entries j0 .. j0 + nr - 1 of
// the span list, nr <= 64: lane l holds span j0 + l (first code, voxel
// offset).  A step is kEmitSlices slices of 256 consecutive codes, 4 per
// lane.  One uniform walk over the spans starting inside the step gives each
// lane the voxel of the first code of each of its quads, and flags quads
// that a span start splits.  An unsplit quad is one 16-byte load; all loads
// of a step are issued before any use; codes are stored 4 at a time
// (aligned: chunks start at multiples of kEmitChunk codes).
template <typename T, int B>
__device__ __forceinline__ void emit_chunk_fast(const T* __restrict__ in, int64_t nx, const Layout& L,
                                                const EmitOut& o, uint64_t c0, uint64_t c1, uint32_t j0, uint32_t nr,
                                                bool& trunc) {
    using C = typename CodeT<B>::type;
    const DevState* S = L.S;
    const int lane = threadIdx.x % kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    const uint32_t esc = S->esc;
    C* codes = reinterpret_cast<C*>(o.stream);
    const bool fits = c1 * (uint64_t)B <= o.stream_cap;
    uint32_t rid = 0;
    uint64_t code0 = ~0ull, off = 0;
    if ((uint32_t)lane < nr) {
        rid = L.nz_rows[j0 + lane];
        code0 = L.row_packed[rid] & kLenMask;
        off = row_origin(L, rid, nx) + L.row_xs[rid] - code0;  // value index = code + off
    }
    constexpr uint32_t kStep = (uint32_t)kEmitSlice * kEmitSlices;
    uint32_t jr = 0;  // span holding the step's first code (uniform)
    for (int s = 0; s < kEmitSteps; ++s) {
        const uint64_t tb = c0 + (uint64_t)s * kStep;
        const uint64_t t0 = tb + 4 * lane;  // first code of this lane's quad in slice 0
        const uint32_t jr_step = jr;
        uint64_t ok[kEmitSlices];
        uint32_t split = 0;
        {
            const uint64_t o0 = readlane64(off, jr);
#pragma unroll
            for (int k = 0; k < kEmitSlices; ++k) ok[k] = o0;
        }
        for (uint32_t jj = jr + 1; jj < nr; ++jj) {
            const uint64_t nc0 = readlane64(code0, jj);
            if (nc0 >= tb + kStep) break;
            const uint64_t on = readlane64(off, jj);
#pragma unroll
            for (int k = 0; k < kEmitSlices; ++k) {
                const uint64_t t = t0 + (uint64_t)k * kEmitSlice;
                if (t >= nc0)
                    ok[k] = on;
                else if (t + 3 >= nc0)
                    split |= 1u << k;
            }
            jr = jj;
        }
        float xv[kEmitSlices][4];
#pragma unroll
        for (int k = 0; k < kEmitSlices; ++k) {
            const uint64_t t = t0 + (uint64_t)k * kEmitSlice;
            if (!((split >> k) & 1u) && t + 3 < c1 && t + ok[k] + quad_reach<T>() <= o.nvox) {
                load_quad(in, t + ok[k], xv[k]);
            } else {
                // a span starts inside this quad (or the chunk ends in it):
                // per-code voxels from the same walk (readlane ignores exec)
                uint64_t vj[4];
                const uint64_t o0 = readlane64(off, jr_step);
#pragma unroll
                for (int j = 0; j < 4; ++j) vj[j] = t + j + o0;
                for (uint32_t jj = jr_step + 1; jj < nr; ++jj) {
                    const uint64_t nc0 = readlane64(code0, jj);
                    if (nc0 >= tb + kStep) break;
                    const uint64_t on = readlane64(off, jj);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (t + j >= nc0) vj[j] = t + j + on;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) xv[k][j] = t + j < c1 ? (float)ld_stream(in + vj[j]) : 0.0f;
            }
        }
        uint32_t anyout = 0;
        uint32_t outm[kEmitSlices];
#pragma unroll
        for (int k = 0; k < kEmitSlices; ++k) {
            const uint64_t t = t0 + (uint64_t)k * kEmitSlice;
            uint32_t u[4];
            uint32_t om = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float x = xv[k][j];
                const int32_t q = qcode(x, r);
                const bool ob = t + j < c1 && outlier(x, q, w, eb32);
                om |= ob ? (1u << j) : 0u;
                u[j] = ob ? esc : (uint32_t)(q - qmin);
            }
            outm[k] = om;
            anyout |= om;
            if (t + 3 < c1 && (fits || (t + 4) * (uint64_t)B <= o.stream_cap)) {
                store_quad<B>(o.stream, t, u);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (t + j >= c1) continue;
                    if ((t + j + 1) * (uint64_t)B <= o.stream_cap)
                        codes[t + j] = (C)u[j];
                    else
                        trunc = true;
                }
            }
        }
        if (__ballot(anyout != 0)) {  // rare: count the step's outliers per span
            for (uint32_t jj = jr_step; jj < nr; ++jj) {
                const uint64_t cj = readlane64(code0, jj);
                if (cj >= tb + kStep) break;
                const uint64_t cn = jj + 1 < nr ? readlane64(code0, jj + 1) : ~0ull;
                uint32_t n = 0;
                for (int k = 0; k < kEmitSlices; ++k) {
                    const uint64_t t = t0 + (uint64_t)k * kEmitSlice;
                    for (int j = 0; j < 4; ++j)
                        n += (uint32_t)__popcll(__ballot(((outm[k] >> j) & 1u) && t + j >= cj && t + j < cn));
                }
                if (n && lane == 0)
                    atomicAdd((unsigned long long*)&L.row_outl[__builtin_amdgcn_readlane(rid, jj)],
                              (unsigned long long)n);
            }
        }
    }
}

__device__ __forceinline__ uint32_t shfl32(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src); }
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = shfl32((uint32_t)v, src), hi = shfl32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// The last lane whose span starts at or before window-relative code `rel`
// (starts increase over the lanes; lanes past the window hold kNone).  Six
// cross-lane reads; every lane of the wave must execute it.
__device__ __forceinline__ int span_lane(uint32_t rs, uint32_t rel) {
    int pos = 0;
#pragma unroll
    for (int st = 32; st > 0; st >>= 1)
        if (shfl32(rs, pos + st) <= rel) pos += st;
    return pos;
}

constexpr int kFastSpans = 16;  // chunks touching more spans take emit_chunk_many
constexpr int kManyQuads = 4;   // quads per lane and round in emit_chunk_many

// Chunks of short spans.  The spans are taken 64 at a time (a window, lane l
// holding span jw + l); the window covers the codes from its first span's
// start to its last span's end.  Each lane takes quads of 4 consecutive
// codes; a binary search over the lanes' span starts gives a quad's span,
// and a quad inside one span is one 16-byte load.  Quads that a span start
// splits, or that the window's ends cut, go code by code.
template <typename T, int B>
__device__ __forceinline__ void emit_chunk_many(const T* __restrict__ in, int64_t nx, const Layout& L,
                                                const EmitOut& o, uint64_t c0, uint64_t c1, uint32_t j0, uint32_t j1,
                                                bool& trunc) {
    using C = typename CodeT<B>::type;
    constexpr int U = kManyQuads;
    const DevState* S = L.S;
    const int lane = threadIdx.x % kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    const uint32_t esc = S->esc;
    C* codes = reinterpret_cast<C*>(o.stream);
    const bool fits = c1 * (uint64_t)B <= o.stream_cap;
    for (uint32_t jw = j0; jw <= j1; jw += kWave) {
        const uint32_t nw = j1 - jw + 1 < (uint32_t)kWave ? j1 - jw + 1 : (uint32_t)kWave;
        uint32_t rid = 0;
        uint64_t cs = ~0ull, ce = 0, off = 0;
        if ((uint32_t)lane < nw) {
            rid = L.nz_rows[jw + lane];
            const uint32_t xs = L.row_xs[rid], xe = L.row_xe[rid];
            cs = L.row_packed[rid] & kLenMask;
            ce = cs + (xe - xs);
            off = row_origin(L, rid, nx) + xs - cs;  // value index = code + off
        }
        const uint64_t cs0 = readlane64(cs, 0);
        const uint64_t wlo = cs0 > c0 ? cs0 : c0;
        const uint64_t cel = readlane64(ce, nw - 1);
        const uint64_t whi = cel < c1 ? cel : c1;
        if (whi <= wlo) continue;
        const uint32_t rs = (uint32_t)lane >= nw ? kNone : (cs <= wlo ? 0u : (uint32_t)(cs - wlo));
        for (uint64_t tq = wlo & ~3ull; tq < whi; tq += 4ull * kWave * U) {
            float x[U][4];
            bool full[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t t = tq + 4ull * (uint64_t)(u * kWave + lane);
                const uint32_t rel = t > wlo ? (uint32_t)(t - wlo) : 0u;
                // span of the quad's first code, and the next three span starts
                // (a span holds at least one code, so a quad meets at most four)
                const int p0 = span_lane(rs, rel);
                uint32_t sn[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const uint32_t v = shfl32(rs, p0 + 1 + k < kWave ? p0 + 1 + k : kWave - 1);
                    sn[k] = p0 + 1 + k < kWave ? v : kNone;
                }
                uint64_t oc[4];
                bool vc[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t c = t + j;
                    const uint32_t rj = c > wlo ? (uint32_t)(c - wlo) : 0u;
                    const int pj = p0 + (sn[0] <= rj) + (sn[1] <= rj) + (sn[2] <= rj);
                    oc[j] = shfl64(off, pj);
                    vc[j] = c >= wlo && c < whi;
                }
                full[u] = vc[0] && vc[3] && sn[0] > rel + 3 && t + oc[0] + quad_reach<T>() <= o.nvox;
                if (full[u]) {
                    load_quad(in, t + oc[0], x[u]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[u][j] = vc[j] ? (float)ld_stream(in + (t + j + oc[j])) : 0.0f;
                }
            }
            uint32_t outm[U];
            uint32_t anyout = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t t = tq + 4ull * (uint64_t)(u * kWave + lane);
                uint32_t cu[4];
                uint32_t om = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float xv = x[u][j];
                    const int32_t q = qcode(xv, r);
                    const bool valid = full[u] || (t + j >= wlo && t + j < whi);
                    const bool ob = valid && outlier(xv, q, w, eb32);
                    om |= ob ? (1u << j) : 0u;
                    cu[j] = ob ? esc : (uint32_t)(q - qmin);
                }
                outm[u] = om;
                anyout |= om;
                if (full[u] && (fits || (t + 4) * (uint64_t)B <= o.stream_cap)) {
                    store_quad<B>(o.stream, t, cu);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint64_t c = t + j;
                        if (c < wlo || c >= whi) continue;
                        if ((c + 1) * (uint64_t)B <= o.stream_cap)
                            codes[c] = (C)cu[j];
                        else
                            trunc = true;
                    }
                }
            }
            if (__ballot(anyout != 0)) {  // rare: per-span outlier counts
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t t = tq + 4ull * (uint64_t)(u * kWave + lane);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint64_t c = t + j;
                        const uint32_t rel = c > wlo ? (uint32_t)(c - wlo) : 0u;
                        const uint32_t rc = shfl32(rid, span_lane(rs, rel));
                        if ((outm[u] >> j) & 1u) atomicAdd((unsigned long long*)&L.row_outl[rc], 1ull);
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Chunks of few spans (the common case of long rows) whose voxels lie within
// 2^30 of the voxel V0 of the chunk's first code: every index is a 32-bit
// byte offset from a uniform base (voxel = V0 + t + d of the code's span, t
// the code's offset in the chunk), so loads and stores take the scalar-base +
// 32-bit offset form.  Lane l < nr holds span l's start rs (0 for a span
// begun before the chunk) and offset d.  Per slice of 256 codes the spans
// are found by a uniform walk over the span starts: a slice without a start
// is one span for every lane, and each start inside a slice costs every
// lane one compare and select per code.  All loads of a step are issued
// before any use.
template <typename T, int B>
__device__ __forceinline__ void store_codes4(uint8_t* dst, const uint32_t (&u)[4]) {
    if constexpr (B == 1) {
        *reinterpret_cast<uint32_t*>(dst) = u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24);
    } else if constexpr (B == 2) {
        *reinterpret_cast<uint2*>(dst) = make_uint2(u[0] | (u[1] << 16), u[2] | (u[3] << 16));
    } else {
        *reinterpret_cast<uint4*>(dst) = make_uint4(u[0], u[1], u[2], u[3]);
    }
}

template <typename T, int B>
__device__ __forceinline__ void emit_chunk_near(const T* __restrict__ in, const Layout& L, const EmitOut& o,
                                                uint64_t c0, uint32_t n, uint32_t nr, uint32_t rs, uint32_t d,
                                                uint32_t rid, uint64_t V0, bool& trunc) {
    using C = typename CodeT<B>::type;
    const DevState* S = L.S;
    const int lane = threadIdx.x % kWave;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    const uint32_t esc = S->esc;
    const uint8_t* base = reinterpret_cast<const uint8_t*>(in + V0);
    const uint64_t vlim64 = o.nvox - V0;  // voxels from V0 to the end of the input
    const uint32_t vlim = uni(vlim64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)vlim64);
    uint8_t* cbase = o.stream + c0 * B;
    const uint64_t cap = o.stream_cap / B;  // codes the stream holds
    const uint32_t nfit = uni(cap <= c0 ? 0u : (cap - c0 >= n ? n : (uint32_t)(cap - c0)));
    constexpr uint32_t kStep = (uint32_t)kEmitSlice * kEmitSlices;
    constexpr uint32_t S_ = (uint32_t)sizeof(T);
    // a whole-quad load reads quad_reach voxels; a volume too short for one
    // at V0 takes the code-by-code loads only
    const bool quads = vlim >= (uint32_t)quad_reach<T>();
    // slice table (lane k: slice k of the chunk): the span of the slice's
    // first code and its offset, and the mask of slices inside which another
    // span starts
    uint32_t jkv = 0;
    bool hk = false;
    {
        const uint32_t tk = (uint32_t)lane * (uint32_t)kEmitSlice;
        for (uint32_t j = 1; j < nr; j = uni(j + 1)) {
            const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
            jkv += sj <= tk ? 1u : 0u;
            hk = hk || (sj > tk && sj < tk + (uint32_t)kEmitSlice);
        }
    }
    const uint32_t dkv = shfl32(d, (int)jkv);  // every lane executes it (jkv < nr <= 64)
    const uint32_t hmask = (uint32_t)__ballot(hk);
    for (uint32_t s0 = 0; s0 < n; s0 += kStep) {
        float xv[kEmitSlices][4];
        uint32_t split = 0;  // slices whose quad is not one contiguous load for some lane
        // phase 1: one quad load per lane and slice, no branches (a split quad
        // loads from voxel V0 and is redone in phase 2), so that every load of
        // the step is in flight before any wait
#pragma unroll
        for (int k = 0; k < kEmitSlices; ++k) {
            const uint32_t tk0 = s0 + (uint32_t)k * kEmitSlice;
            const uint32_t t = tk0 + 4u * (uint32_t)lane;
            const uint32_t kk = tk0 / (uint32_t)kEmitSlice;
            const uint32_t dc = uni(__builtin_amdgcn_readlane(dkv, kk));
            uint32_t d0 = dc, d3 = dc;
            if ((hmask >> kk) & 1u) {  // uniform: starts inside this slice
                for (uint32_t j = uni(__builtin_amdgcn_readlane(jkv, kk)) + 1; j < nr; j = uni(j + 1)) {
                    const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
                    if (sj >= tk0 + (uint32_t)kEmitSlice) break;
                    const uint32_t dj = uni(__builtin_amdgcn_readlane(d, j));
                    d0 = t >= sj ? dj : d0;
                    d3 = t + 3 >= sj ? dj : d3;
                }
            }
            const bool full = quads && t + 4 <= n && d0 == d3 && t + d0 + (uint32_t)quad_reach<T>() <= vlim;
            if (__ballot(!full)) split |= 1u << k;
            const uint32_t vi = full ? t + d0 : 0u;  // voxels V0 .. V0 + quad_reach - 1 exist when quads holds
            if (!quads) {  // uniform
#pragma unroll
                for (int i = 0; i < 4; ++i) xv[k][i] = 0.0f;
            } else if constexpr (sizeof(T) == 4) {
                const v4u32_t q = *(reinterpret_cast<const v4u32_t*>(base + vi * S_));
                xv[k][0] = __uint_as_float(q.x);
                xv[k][1] = __uint_as_float(q.y);
                xv[k][2] = __uint_as_float(q.z);
                xv[k][3] = __uint_as_float(q.w);
            } else {
                load_quad(in, V0 + (uint64_t)vi, xv[k]);
            }
        }
        // phase 2: the split quads, code by code (slices with span starts, the chunk's end)
        if (split) {
#pragma unroll
            for (int k = 0; k < kEmitSlices; ++k) {
                if (!((split >> k) & 1u)) continue;  // uniform
                const uint32_t tk0 = s0 + (uint32_t)k * kEmitSlice;
                const uint32_t t = tk0 + 4u * (uint32_t)lane;
                const uint32_t kk = tk0 / (uint32_t)kEmitSlice;
                const uint32_t dc = uni(__builtin_amdgcn_readlane(dkv, kk));
                uint32_t di[4] = {dc, dc, dc, dc};
                if ((hmask >> kk) & 1u) {
                    for (uint32_t j = uni(__builtin_amdgcn_readlane(jkv, kk)) + 1; j < nr; j = uni(j + 1)) {
                        const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
                        if (sj >= tk0 + (uint32_t)kEmitSlice) break;
                        const uint32_t dj = uni(__builtin_amdgcn_readlane(d, j));
#pragma unroll
                        for (int i = 0; i < 4; ++i) di[i] = t + (uint32_t)i >= sj ? dj : di[i];
                    }
                }
                const bool full =
                    quads && t + 4 <= n && di[0] == di[3] && t + di[0] + (uint32_t)quad_reach<T>() <= vlim;
                if (!full) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        xv[k][i] = t + (uint32_t)i < n ? (float)ld_stream(reinterpret_cast<const T*>(
                                                             base + (t + (uint32_t)i + di[i]) * S_))
                                                       : 0.0f;
                }
            }
        }
        // phase 3: codes.  A slice wholly inside the chunk and the stream needs
        // no per-code checks.
        uint32_t outm[kEmitSlices];
        uint32_t anyout = 0;
#pragma unroll
        for (int k = 0; k < kEmitSlices; ++k) {
            const uint32_t tk0 = s0 + (uint32_t)k * kEmitSlice;
            const uint32_t t = tk0 + 4u * (uint32_t)lane;
            uint32_t u[4];
            uint32_t om = 0;
            if (tk0 + (uint32_t)kEmitSlice <= nfit) {  // uniform
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x = xv[k][i];
                    const int32_t q = qcode(x, r);
                    const bool ob = outlier(x, q, w, eb32);
                    om |= ob ? (1u << i) : 0u;
                    u[i] = ob ? esc : (uint32_t)(q - qmin);
                }
                store_codes4<T, B>(cbase + t * B, u);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x = xv[k][i];
                    const int32_t q = qcode(x, r);
                    const bool ob = t + (uint32_t)i < n && outlier(x, q, w, eb32);
                    om |= ob ? (1u << i) : 0u;
                    u[i] = ob ? esc : (uint32_t)(q - qmin);
                }
                if (t + 4 <= nfit) {
                    store_codes4<T, B>(cbase + t * B, u);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (t + (uint32_t)i >= n) continue;
                        if (t + (uint32_t)i < nfit)
                            reinterpret_cast<C*>(cbase + t * B)[i] = (C)u[i];
                        else
                            trunc = true;
                    }
                }
            }
            outm[k] = om;
            anyout |= om;
        }
        if (__ballot(anyout != 0)) {  // rare: per-span outlier counts
#pragma unroll
            for (int k = 0; k < kEmitSlices; ++k) {
                const uint32_t t = s0 + (uint32_t)k * kEmitSlice + 4u * (uint32_t)lane;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int jj = 0;
                    for (uint32_t j = 1; j < nr; j = uni(j + 1))
                        jj = t + (uint32_t)i >= uni(__builtin_amdgcn_readlane(rs, j)) ? (int)j : jj;
                    const uint32_t rc = shfl32(rid, jj);  // every lane executes it
                    if ((outm[k] >> i) & 1u) atomicAdd((unsigned long long*)&L.row_outl[rc], 1ull);
                }
            }
        }
    }
}

// Near chunks read from the 16-bit proxy of the fused pass (float32 volumes
// whose rows are whole 64-voxel words, so that proxy element = voxel): the
// proxy holds q mod 2^15 and the outlier flag, so a code is
// q - qmin = (p - qmin) mod 2^15, or the escape for a flagged voxel, and
// emitting needs no quantiser arithmetic and half the input bytes.  Lane l
// takes codes 8 l .. 8 l + 7 of each 512-code slice.  Codes of one span are
// one 16-byte load from the 4-byte-aligned element at or before the first
// (plus the next dword, funnel-shifted in, when that element is odd); in a
// slice where spans start, a second such load at the offset of the lane's
// last code covers a lane whose codes cross one span start, and phase 3
// picks each code from the load of its span.  Lanes with codes of three or
// more spans, at the chunk's end or at the end of the proxy store whatever
// phase 3 makes of their stand-in loads and then redo their codes one by one
// (phase 4).  Slice table and span walk as in emit_chunk_near, with 512-code
// slices.
constexpr uint32_t kP16Slice = 512;
constexpr int kP16Slices = 2;  // slices per step

__device__ __forceinline__ uint32_t half16(const uint32_t (&w)[4], int i) { return (w[i >> 1] >> (16 * (i & 1))) & 0xFFFFu; }

// 8 elements from a whole load (4 dwords + the next) shifted by sh bits
__device__ __forceinline__ void funnel8(const uint32_t (&a)[5], uint32_t sh, uint32_t (&w)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_alignbit(a[i + 1], a[i], sh);
}

// VALS: px is a uint16 volume (element = voxel for any row width) and each
// code comes from the quantiser, as in emit_chunk_near, on the same loads.
template <int B, bool VALS = false>
__device__ __forceinline__ void emit_chunk_p16(const uint16_t* __restrict__ px, const Layout& L, const EmitOut& o,
                                               uint64_t c0, uint32_t n, uint32_t nr, uint32_t rs, uint32_t d,
                                               uint32_t rid, uint64_t V0, bool& trunc) {
    using C = typename CodeT<B>::type;
    const DevState* S = L.S;
    const int lane = threadIdx.x % kWave;
    const uint32_t Q2 = ((uint32_t)S->qmin & 0x7FFFu) * 0x00010001u;
    const uint32_t esc = S->esc;
    const float qr = S->r, qw = S->w, eb32 = S->eb32;
    const int32_t qmin = S->qmin;
    // the code of value p and whether p is an outlier
    auto vcode = [&](uint32_t p, bool& ob) -> uint32_t {
        const float x = (float)p;
        const int32_t q = qcode(x, qr);
        ob = outlier(x, q, qw, eb32);
        return ob ? esc : (uint32_t)(q - qmin);
    };
    const uint16_t* base = px + V0;
    const uint64_t vlim64 = o.nvox - V0;  // elements from V0 to the end of the proxy
    const uint32_t vlim = uni(vlim64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)vlim64);
    uint8_t* cbase = o.stream + c0 * B;
    const uint64_t cap = o.stream_cap / B;
    const uint32_t nfit = uni(cap <= c0 ? 0u : (cap - c0 >= n ? n : (uint32_t)(cap - c0)));
    constexpr uint32_t kStep = kP16Slice * kP16Slices;
    // a whole load at offset v reads elements v - 1 .. v + 9 at most, so it
    // needs v + 10 <= vlim; a proxy too short for one at V0 goes code by code
    const bool whole = vlim >= 10u;
    const uint32_t odd0 = (uint32_t)(V0 & 1ull);
    uint32_t jkv = 0;
    bool hk = false;
    {
        const uint32_t tk = (uint32_t)lane * kP16Slice;
        for (uint32_t j = 1; j < nr; j = uni(j + 1)) {
            const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
            jkv += sj <= tk ? 1u : 0u;
            hk = hk || (sj > tk && sj < tk + kP16Slice);
        }
    }
    const uint32_t dkv = shfl32(d, (int)jkv);  // every lane executes it (jkv < nr <= 64)
    const uint32_t hmask = (uint32_t)__ballot(hk);
    for (uint32_t s0 = 0; s0 < n; s0 += kStep) {
        uint32_t la[kP16Slices][5], lb[kP16Slices][5], sa[kP16Slices], sb[kP16Slices], cut[kP16Slices];
        uint32_t split = 0, bad = 0;
        // phase 1: every load of the step, no lane branches (a lane that
        // cannot take whole loads loads at V0 and is redone in phase 4)
#pragma unroll
        for (int k = 0; k < kP16Slices; ++k) {
            const uint32_t tk0 = s0 + (uint32_t)k * kP16Slice;
            const uint32_t t = tk0 + 8u * (uint32_t)lane;
            const uint32_t kk = tk0 / kP16Slice;
            const uint32_t dc = uni(__builtin_amdgcn_readlane(dkv, kk));
            const bool starts = (hmask >> kk) & 1u;  // uniform
            uint32_t d0 = dc, d7 = dc, i0 = 8u;
            bool multi = false;
            if (starts) {
                for (uint32_t j = uni(__builtin_amdgcn_readlane(jkv, kk)) + 1; j < nr; j = uni(j + 1)) {
                    const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
                    if (sj >= tk0 + kP16Slice) break;
                    const uint32_t dj = uni(__builtin_amdgcn_readlane(d, j));
                    const bool inside = sj > t && sj <= t + 7;
                    multi = multi || (inside && i0 != 8u);
                    i0 = (inside && i0 == 8u) ? sj - t : i0;
                    d0 = t >= sj ? dj : d0;
                    d7 = t + 7 >= sj ? dj : d7;
                }
            }
            const uint32_t va = t + d0, vb = t + d7;  // vb >= va: offsets never decrease
            const bool full = whole && t + 8 <= n && !multi && vb + 10 <= vlim;
            if (__ballot(!full)) split |= 1u << k;
            bad |= full ? 0u : (1u << k);
            cut[k] = i0;
            const uint32_t oa = full ? ((odd0 + va) & 1u) : odd0;
            const int64_t aa = full ? (int64_t)va - (int64_t)oa : -(int64_t)odd0;
            sa[k] = 16u * oa;
            if (whole) {  // uniform; elements V0 - odd0 .. V0 - odd0 + 9 exist
                const v4u32_t q = *(reinterpret_cast<const v4u32_t*>(base + aa));
                la[k][0] = q.x;
                la[k][1] = q.y;
                la[k][2] = q.z;
                la[k][3] = q.w;
                la[k][4] = *(reinterpret_cast<const uint32_t*>(base + aa + 8));
                if (starts) {
                    const uint32_t ob = full ? ((odd0 + vb) & 1u) : odd0;
                    const int64_t ab = full ? (int64_t)vb - (int64_t)ob : -(int64_t)odd0;
                    sb[k] = 16u * ob;
                    const v4u32_t r = *(reinterpret_cast<const v4u32_t*>(base + ab));
                    lb[k][0] = r.x;
                    lb[k][1] = r.y;
                    lb[k][2] = r.z;
                    lb[k][3] = r.w;
                    lb[k][4] = *(reinterpret_cast<const uint32_t*>(base + ab + 8));
                }
            } else {
#pragma unroll
                for (int i = 0; i < 5; ++i) la[k][i] = 0u;
            }
        }
        // phase 3: codes
        uint32_t outm[kP16Slices];
        uint32_t anyout = 0;
#pragma unroll
        for (int k = 0; k < kP16Slices; ++k) {
            const uint32_t tk0 = s0 + (uint32_t)k * kP16Slice;
            const uint32_t t = tk0 + 8u * (uint32_t)lane;
            uint32_t w[4];
            funnel8(la[k], sa[k], w);
            if ((hmask >> (tk0 / kP16Slice)) & 1u) {  // uniform: codes from cut on come from the second load
                uint32_t wb[4];
                funnel8(lb[k], sb[k], wb);
                const uint32_t c8 = cut[k];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t keep = c8 >= 2u * i + 2u ? 0xFFFFFFFFu : (c8 == 2u * i + 1u ? 0x0000FFFFu : 0u);
                    w[i] = (w[i] & keep) | (wb[i] & ~keep);
                }
            }
            uint32_t c[4], om = 0;
            if constexpr (VALS) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    bool o0, o1;
                    const uint32_t u0 = vcode(w[i] & 0xFFFFu, o0), u1 = vcode(w[i] >> 16, o1);
                    c[i] = u0 | (u1 << 16);
                    om |= (o0 ? 1u : 0u) << (2 * i);
                    om |= (o1 ? 1u : 0u) << (2 * i + 1);
                }
                if ((bad >> k) & 1u) om = 0;  // a lane that phase 4 redoes
            } else {
                uint32_t fl = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fl |= w[i] & 0x80008000u;
                    c[i] = ((w[i] | 0x80008000u) - Q2) & 0x7FFF7FFFu;
                }
                // flag bits of codes 0..7 (none for a lane that phase 4 redoes)
                if (fl && !((bad >> k) & 1u)) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) om |= ((half16(w, i) >> 15) & 1u) << i;
                }
            }
            if (tk0 + kP16Slice <= nfit) {  // uniform: the slice lies inside the chunk and the stream
                if constexpr (B == 2) {
                    *reinterpret_cast<uint4*>(cbase + 2 * t) = make_uint4(c[0], c[1], c[2], c[3]);
                } else {
                    uint32_t b[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) b[i] = (c[i] & 0xFFu) | ((c[i] >> 8) & 0xFF00u);
                    *reinterpret_cast<uint2*>(cbase + t) = make_uint2(b[0] | (b[1] << 16), b[2] | (b[3] << 16));
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (t + (uint32_t)i >= n) continue;
                    if (t + (uint32_t)i < nfit)
                        reinterpret_cast<C*>(cbase + (uint64_t)t * B)[i] = (C)half16(c, i);
                    else
                        trunc = true;
                }
            }
            outm[k] = om;
            anyout |= om;
        }
        if (__ballot(anyout != 0)) {  // rare: escapes and per-span outlier counts
#pragma unroll
            for (int k = 0; k < kP16Slices; ++k) {
                const uint32_t t = s0 + (uint32_t)k * kP16Slice + 8u * (uint32_t)lane;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int jj = 0;
                    for (uint32_t j = 1; j < nr; j = uni(j + 1))
                        jj = t + (uint32_t)i >= uni(__builtin_amdgcn_readlane(rs, j)) ? (int)j : jj;
                    const uint32_t rc = shfl32(rid, jj);  // every lane executes it
                    if ((outm[k] >> i) & 1u) {
                        atomicAdd((unsigned long long*)&L.row_outl[rc], 1ull);
                        if (t + (uint32_t)i < nfit) reinterpret_cast<C*>(cbase + (uint64_t)t * B)[i] = (C)esc;
                    }
                }
            }
        }
        // phase 4 (rare): the lanes marked bad, code by code over their own
        // stores (same lane, program order)
        if (split) {
#pragma unroll
            for (int k = 0; k < kP16Slices; ++k) {
                if (!((split >> k) & 1u)) continue;  // uniform
                const uint32_t tk0 = s0 + (uint32_t)k * kP16Slice;
                const uint32_t t = tk0 + 8u * (uint32_t)lane;
                const uint32_t kk = tk0 / kP16Slice;
                const uint32_t dc = uni(__builtin_amdgcn_readlane(dkv, kk));
                uint32_t di[8] = {dc, dc, dc, dc, dc, dc, dc, dc};
                int ji[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // span (lane of rid) of each code
                const int jc = (int)uni(__builtin_amdgcn_readlane(jkv, kk));
#pragma unroll
                for (int i = 0; i < 8; ++i) ji[i] = jc;
                if ((hmask >> kk) & 1u) {
                    for (uint32_t j = (uint32_t)jc + 1; j < nr; j = uni(j + 1)) {
                        const uint32_t sj = uni(__builtin_amdgcn_readlane(rs, j));
                        if (sj >= tk0 + kP16Slice) break;
                        const uint32_t dj = uni(__builtin_amdgcn_readlane(d, j));
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const bool in = t + (uint32_t)i >= sj;
                            di[i] = in ? dj : di[i];
                            ji[i] = in ? (int)j : ji[i];
                        }
                    }
                }
                const bool redo = (bad >> k) & 1u;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t rc = shfl32(rid, ji[i]);  // every lane executes it
                    if (!redo || t + (uint32_t)i >= n) continue;
                    const uint32_t p = (uint32_t)ld_stream(base + (t + (uint32_t)i + di[i]));
                    bool ob;
                    uint32_t code;
                    if constexpr (VALS) {
                        code = vcode(p, ob);
                    } else {
                        ob = (p >> 15) & 1u;
                        code = ob ? esc : ((p | 0x8000u) - (Q2 & 0xFFFFu)) & 0x7FFFu;
                    }
                    if (ob) atomicAdd((unsigned long long*)&L.row_outl[rc], 1ull);
                    if (t + (uint32_t)i < nfit)
                        reinterpret_cast<C*>(cbase + (uint64_t)t * B)[i] = (C)code;
                    else
                        trunc = true;
                }
            }
        }
    }
}

// Chunk q's bounds and span range (uniform).
__device__ __forceinline__ void chunk_of(const Layout& L, uint64_t q, uint64_t nchunks, uint64_t n_codes,
                                         uint32_t n_rows, uint64_t& c0, uint64_t& c1, uint32_t& j0, uint32_t& j1) {
    c0 = q * kEmitChunk;
    c1 = c0 + kEmitChunk < n_codes ? c0 + kEmitChunk : n_codes;
    j0 = uni(L.chunk_row[q]);
    j1 = uni(q + 1 < nchunks ? L.chunk_row[q + 1] : n_rows - 1);
}

// The codes of every span voxel, in row order, as one flat stream: each wave
// takes whole kEmitChunk-code chunks, so loads and stores are contiguous and
// no lane idles on a short row.  The lean path takes chunks of at most 64
// spans (one per lane) within 2^30 voxels and queues every other chunk for
// the general kernel, so that its register budget stays that of the lean
// path.  B = bytes per code.
template <typename T, int B, bool P16 = false, bool VALS = false>
__device__ __forceinline__ void emit_codes_lean(const VPart vp, const T* __restrict__ in, int64_t nx, const Layout& L,
                                                const EmitOut& o, const uint16_t* __restrict__ px = nullptr) {
    DevState* S = L.S;
    bool trunc = false;
    const uint64_t n_codes = uni64(S->span_total & kLenMask);
    const uint32_t n_rows = uni((uint32_t)(S->span_total >> 40));
    const uint64_t nchunks = (n_codes + kEmitChunk - 1) / kEmitChunk;
    const int lane = threadIdx.x % kWave;
    const uint64_t wave = uni((vp.b * blockDim.x + threadIdx.x) / kWave);
    const uint64_t nwaves = (uint64_t)vp.n * blockDim.x / kWave;
    for (uint64_t q = wave; q < nchunks; q += nwaves) {
        uint64_t c0, c1;
        uint32_t j0, j1;
        chunk_of(L, q, nchunks, n_codes, n_rows, c0, c1, j0, j1);
        const uint32_t nr = j1 - j0 + 1;
        bool near = false;
        uint32_t rid = 0, rs = kNone, d = 0;
        uint64_t off0 = 0;
        if (nr <= (uint32_t)kWave) {
            uint64_t cs = ~0ull, off = 0;
            if ((uint32_t)lane < nr) {
                const uint4 sd = *reinterpret_cast<const uint4*>(L.span_desc + 2 * (uint64_t)(j0 + lane));
                cs = ((uint64_t)sd.y << 32) | sd.x;
                off = ((uint64_t)sd.w << 32) | sd.z;  // voxel = code + off
                rid = L.nz_rows[j0 + lane];
            }
            // the chunk's voxels are [V0, V0 + (c1 - 1 - c0) + d_last]: offsets
            // never decrease from one span to the next
            off0 = uni64(readlane64(off, 0));
            const uint64_t dl = uni64(readlane64(off, nr - 1)) - off0;
            near = (c1 - 1 - c0) + dl < (1ull << 30);
            rs = (uint32_t)lane >= nr ? kNone : (cs <= c0 ? 0u : (uint32_t)(cs - c0));
            d = (uint32_t)lane >= nr ? 0u : (uint32_t)(off - off0);
        }
        if (near) {
            if constexpr (P16)
                emit_chunk_p16<B, VALS>(px, L, o, c0, (uint32_t)(c1 - c0), nr, rs, d, rid, c0 + off0, trunc);
            else
                emit_chunk_near<T, B>(in, L, o, c0, (uint32_t)(c1 - c0), nr, rs, d, rid, c0 + off0, trunc);
        } else if (lane == 0) {
            L.slow_chunks[atomicAdd(&S->n_slow, 1u)] = (uint32_t)q;
        }
    }
    if (trunc) atomicOr(&S->trunc, 1);
}

// The queued chunks: many short spans (lane windows with a cross-lane
// search), or few spans whose voxels lie far apart (64-bit offsets).  A
// chunk of many spans is shared by kGenSplit waves, each taking a quarter of
// its codes (the lane windows clip to that range), so that a volume with few
// chunks, all of short spans, is not left to a handful of waves.
constexpr uint32_t kGenSplit = 4;
template <typename T, int B>
__device__ __forceinline__ void emit_codes_general(const VPart vp, const T* __restrict__ in, int64_t nx,
                                                   const Layout& L, const EmitOut& o) {
    DevState* S = L.S;
    bool trunc = false;
    const uint64_t n_codes = uni64(S->span_total & kLenMask);
    const uint32_t n_rows = uni((uint32_t)(S->span_total >> 40));
    const uint64_t nchunks = (n_codes + kEmitChunk - 1) / kEmitChunk;
    const uint32_t nq = uni(S->n_slow);
    const uint32_t wave = uni((vp.b * blockDim.x + threadIdx.x) / kWave);
    const uint32_t nwaves = vp.n * blockDim.x / kWave;
    for (uint32_t i = wave; i < nq * kGenSplit; i += nwaves) {
        const uint64_t q = uni(L.slow_chunks[i / kGenSplit]);
        const uint32_t part = i % kGenSplit;
        uint64_t c0, c1;
        uint32_t j0, j1;
        chunk_of(L, q, nchunks, n_codes, n_rows, c0, c1, j0, j1);
        if (j1 - j0 < (uint32_t)kFastSpans) {
            if (part == 0) emit_chunk_fast<T, B>(in, nx, L, o, c0, c1, j0, j1 - j0 + 1, trunc);
        } else {
            const uint64_t a = c0 + (uint64_t)part * (kEmitChunk / kGenSplit);
            const uint64_t b = a + kEmitChunk / kGenSplit < c1 ? a + kEmitChunk / kGenSplit : c1;
            if (a < b) emit_chunk_many<T, B>(in, nx, L, o, a, b, j0, j1, trunc);
        }
    }
    if (trunc) atomicOr(&S->trunc, 1);
}

// The code width is device data (resolved from the value range); the branch
// on it is uniform.  unless_p16: nothing to do when the 16-bit proxy kernel
// below takes the lean chunks.
template <typename T>
__device__ __forceinline__ void k_emit_codes_body(const VPart vp, const T* __restrict__ in, int64_t nx, Layout L, EmitOut o,
                                                       int unless_p16) {
    if (thread_exit_e(L.S)) return;  // no barrier below
    if (unless_p16 && L.S->p16) return;
    const int wb = L.S->width_bits;
    if constexpr (sizeof(T) == 2) {
        // 16-bit values: the 16-bit proxy kernel's loads (8 codes a lane, a
        // 16-byte load and a dword per span), codes from the quantiser
        const uint16_t* v16 = reinterpret_cast<const uint16_t*>(in);
        if (wb == 16)
            emit_codes_lean<T, 2, true, true>(vp, in, nx, L, o, v16);
        else if (wb == 8)
            emit_codes_lean<T, 1, true, true>(vp, in, nx, L, o, v16);
        else
            emit_codes_lean<T, 4>(vp, in, nx, L, o);
        return;
    }
    if (wb == 16)
        emit_codes_lean<T, 2>(vp, in, nx, L, o);
    else if (wb == 8)
        emit_codes_lean<T, 1>(vp, in, nx, L, o);
    else
        emit_codes_lean<T, 4>(vp, in, nx, L, o);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit_codes(const T* __restrict__ in, int64_t nx, Layout L, EmitOut o,
                                                       int unless_p16) {
    k_emit_codes_body<T>(hw_part(), in, nx, L, o, unless_p16);
}

// The lean chunks from the 16-bit proxy, when the fused pass produced it
// (K <= 2^15, so codes are 8 or 16 bits wide).
__device__ __forceinline__ void k_emit_codes_p16_body(const VPart vp, const float* __restrict__ in, int64_t nx, Layout L,
                                                           EmitOut o, const uint16_t* __restrict__ px) {
    if (thread_exit_e(L.S) || !L.S->p16) return;  // no barrier below
    if (L.S->width_bits == 16)
        emit_codes_lean<float, 2, true>(vp, in, nx, L, o, px);
    else
        emit_codes_lean<float, 1, true>(vp, in, nx, L, o, px);
}
// float32 volumes in one launch: the lean chunks from the 16-bit proxy (and
// the image `in`) when the fused pass produced it, else from the values
// `vals` (the image, or M with a background).  The branch is uniform.
__device__ __forceinline__ void k_emit_codes_f32_body(const VPart vp, const float* __restrict__ in,
                                                      const float* __restrict__ vals, int64_t nx, Layout L, EmitOut o,
                                                      const uint16_t* __restrict__ px) {
    if (px && !thread_exit_e(L.S) && L.S->p16)
        k_emit_codes_p16_body(vp, in, nx, L, o, px);
    else
        k_emit_codes_body<float>(vp, vals, nx, L, o, 0);
}
__global__ __launch_bounds__(kBlock) void k_emit_codes_f32(const float* __restrict__ in, const float* __restrict__ vals,
                                                           int64_t nx, Layout L, EmitOut o,
                                                           const uint16_t* __restrict__ px) {
    k_emit_codes_f32_body(hw_part(), in, vals, nx, L, o, px);
}

template <typename T>
__device__ __forceinline__ void k_emit_codes_general_body(const VPart vp, const T* __restrict__ in, int64_t nx, Layout L,
                                                               EmitOut o) {
    if (thread_exit_e(L.S)) return;  // no barrier below
    const int wb = L.S->width_bits;
    if (wb == 16)
        emit_codes_general<T, 2>(vp, in, nx, L, o);
    else if (wb == 8)
        emit_codes_general<T, 1>(vp, in, nx, L, o);
    else
        emit_codes_general<T, 4>(vp, in, nx, L, o);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit_codes_general(const T* __restrict__ in, int64_t nx, Layout L,
                                                               EmitOut o) {
    k_emit_codes_general_body<T>(hw_part(), in, nx, L, o);
}

// Outlier values: a span of up to 1024 voxels is one round of 16 loads per
// lane; the test recomputes the quantiser and the values are stored in order
// of x from the span's outlier offset.
constexpr int kOutlU = 16;  // loads per lane and round
constexpr uint32_t kOutlRound = (uint32_t)kWave * kOutlU;

template <typename T, bool BG = false>
__device__ __forceinline__ void outl_load(const T* __restrict__ src, const float* __restrict__ bsrc, uint32_t len,
                                          uint32_t j0, float (&xv)[kOutlU]) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int u = 0; u < kOutlU; ++u) {
        const uint32_t jj = j0 + u * kWave + lane;
        const uint32_t js = jj < len ? jj : 0u;
        if constexpr (BG)
            xv[u] = (float)src[js] - bsrc[js];  // M = I - B, the value the codes were taken of
        else
            xv[u] = (float)src[js];
    }
}

__device__ __forceinline__ void outl_store(const float (&xv)[kOutlU], uint32_t len, uint32_t j0, float r, float w,
                                           float eb32, unsigned long long& k, const EmitOut& o, bool& trunc) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int u = 0; u < kOutlU; ++u) {
        const uint32_t jj = j0 + u * kWave + lane;
        const float x = xv[u];
        const bool isout = jj < len && outlier(x, qcode(x, r), w, eb32);
        const uint64_t mo = __ballot(isout);
        if (isout) {
            const unsigned long long at = k + (unsigned long long)__popcll(mo & ((1ull << lane) - 1ull));
            if (at < o.outl_cap)
                o.outl[at] = x;
            else
                trunc = true;
        }
        k += (unsigned long long)__popcll(mo);
    }
}

// The 16-bit proxy's outlier flags (bit 15) of one round, and the stores of
// the flagged voxels' values (read from the input, I - B with a background)
// in order of x from the span's outlier offset.
__device__ __forceinline__ void outl_flags(const uint16_t* __restrict__ ps, uint32_t len, uint32_t j0,
                                           uint32_t (&fv)[kOutlU]) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int u = 0; u < kOutlU; ++u) {
        const uint32_t jj = j0 + u * kWave + lane;
        fv[u] = ps[jj < len ? jj : 0u];
    }
}

template <typename T, bool BG>
__device__ __forceinline__ void outl_store_flagged(const uint32_t (&fv)[kOutlU], const T* __restrict__ src,
                                                   const float* __restrict__ bsrc, uint32_t len, uint32_t j0,
                                                   unsigned long long& k, const EmitOut& o, bool& trunc) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int u = 0; u < kOutlU; ++u) {
        const uint32_t jj = j0 + u * kWave + lane;
        const bool isout = jj < len && ((fv[u] >> 15) & 1u);
        const uint64_t mo = __ballot(isout);
        if (isout) {
            float x;
            if constexpr (BG)
                x = (float)src[jj] - bsrc[jj];
            else
                x = (float)src[jj];
            const unsigned long long at = k + (unsigned long long)__popcll(mo & ((1ull << lane) - 1ull));
            if (at < o.outl_cap)
                o.outl[at] = x;
            else
                trunc = true;
        }
        k += (unsigned long long)__popcll(mo);
    }
}

// After the scan of the per-row outlier counts.  Each wave takes 64 spans,
// one per lane: the lane writes its span's row table entry (coalesced), then
// the wave walks the spans that have outliers (a ballot), the first round of
// the next one in flight while the current one is tested.  px: the 16-bit
// proxy (element = voxel), or null; when the call took the one-pass flow the
// outliers are found by its flag bits (2 bytes a voxel) and only their
// values are read from the input.
template <typename T, bool BG = false>
__device__ __forceinline__ void k_emit_rows_body(const VPart vp, const T* __restrict__ in, int64_t nx, Layout L, int64_t ny,
                                                      int64_t nrows, EmitOut o, const float* __restrict__ bg,
                                                      int bg_plane, const uint16_t* __restrict__ px) {
    DevState* S = L.S;
    if (thread_exit_e(S)) return;
    const uint32_t n_rows = uni((uint32_t)(S->span_total >> 40));
    const unsigned long long total = S->n_outliers;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int lane = threadIdx.x % kWave;
    const uint32_t wave = uni((vp.b * blockDim.x + threadIdx.x) / kWave);
    const uint32_t nwaves = vp.n * blockDim.x / kWave;
    bool trunc = false;
    for (uint64_t jb = (uint64_t)wave * kWave; jb < n_rows; jb += (uint64_t)nwaves * kWave) {
        const uint32_t j = (uint32_t)jb + (uint32_t)lane;
        const bool valid = j < n_rows;
        uint32_t rid = 0, xs = 0, len = 0;
        uint64_t ooff = 0, oend = 0;
        if (valid) {
            rid = L.nz_rows[j];
            ooff = L.row_outl[rid];
            oend = (int64_t)rid + 1 < nrows ? L.row_outl[rid + 1] : total;
            xs = L.row_xs[rid];
            const uint32_t xe = L.row_xe[rid];
            len = xe - xs;
            if (j < o.rows_cap) {
                roix_row e;
                e.z = rid / (uint32_t)ny;
                e.y = rid - e.z * (uint32_t)ny;
                e.xs = xs;
                e.xe = xe;
                e.code_off = L.row_packed[rid] & kLenMask;
                e.outlier_off = ooff;
                o.rows[j] = e;
            } else {
                trunc = true;
            }
        }
        uint64_t m = __ballot(valid && oend != ooff);
        if (!m) continue;  // uniform
        auto src_of = [&](int l) {
            return in + uni64(row_origin(L, uni(__builtin_amdgcn_readlane(rid, l)), nx)) +
                   uni(__builtin_amdgcn_readlane(xs, l));
        };
        // the reference row under span l: plane row (row mod ny) or the row itself
        auto bsrc_of = [&](int l) -> const float* {
            if constexpr (!BG) return nullptr;
            const uint64_t rr = (uint64_t)uni(__builtin_amdgcn_readlane(rid, l));
            return bg + (bg_plane ? rr % (uint64_t)ny : rr) * (uint64_t)nx + uni(__builtin_amdgcn_readlane(xs, l));
        };
        auto len_of = [&](int l) { return uni(__builtin_amdgcn_readlane(len, l)); };
        if (px && S->p16) {  // uniform: the proxy's flags, ping-pong over the spans as below
            auto psrc_of = [&](int l) {
                return px + (uint64_t)uni(__builtin_amdgcn_readlane(rid, l)) * (uint64_t)nx +
                       uni(__builtin_amdgcn_readlane(xs, l));
            };
            auto ftest = [&](int l, const uint32_t (&fv)[kOutlU]) {
                const uint32_t lt = len_of(l);
                unsigned long long k = readlane64(ooff, l);
                outl_store_flagged<T, BG>(fv, src_of(l), bsrc_of(l), lt, 0, k, o, trunc);
                for (uint32_t j0 = kOutlRound; j0 < lt; j0 += kOutlRound) {
                    uint32_t fc[kOutlU];
                    outl_flags(psrc_of(l), lt, j0, fc);
                    outl_store_flagged<T, BG>(fc, src_of(l), bsrc_of(l), lt, j0, k, o, trunc);
                }
            };
            auto fpop = [&](int prev) {
                if (!m) return prev;
                const int l = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                return l;
            };
            uint32_t fa[kOutlU], fb[kOutlU];
            int la = fpop(0);
            outl_flags(psrc_of(la), len_of(la), 0, fa);
            while (true) {
                const bool more_b = m != 0;
                const int lb = fpop(la);
                outl_flags(psrc_of(lb), len_of(lb), 0, fb);
                ftest(la, fa);
                if (!more_b) break;
                const bool more_a = m != 0;
                la = fpop(lb);
                outl_flags(psrc_of(la), len_of(la), 0, fa);
                ftest(lb, fb);
                if (!more_a) break;
            }
            continue;
        }
        // one span: its first round is in xv; longer spans loop (rare)
        auto test = [&](int l, const float (&xv)[kOutlU]) {
            const uint32_t lt = len_of(l);
            unsigned long long k = readlane64(ooff, l);
            outl_store(xv, lt, 0, r, w, eb32, k, o, trunc);
            for (uint32_t j0 = kOutlRound; j0 < lt; j0 += kOutlRound) {
                float xc[kOutlU];
                outl_load<T, BG>(src_of(l), bsrc_of(l), lt, j0, xc);
                outl_store(xc, lt, j0, r, w, eb32, k, o, trunc);
            }
        };
        // ping-pong over the spans with outliers; past the last one the
        // loads repeat it (harmless), so every load is unconditional
        auto pop = [&](int prev) {
            if (!m) return prev;
            const int l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            return l;
        };
        float xa[kOutlU], xb[kOutlU];
        int la = pop(0);
        outl_load<T, BG>(src_of(la), bsrc_of(la), len_of(la), 0, xa);
        while (true) {
            const bool more_b = m != 0;
            const int lb = pop(la);
            outl_load<T, BG>(src_of(lb), bsrc_of(lb), len_of(lb), 0, xb);
            test(la, xa);
            if (!more_b) break;
            const bool more_a = m != 0;
            la = pop(lb);
            outl_load<T, BG>(src_of(la), bsrc_of(la), len_of(la), 0, xa);
            test(lb, xb);
            if (!more_a) break;
        }
    }
    if (trunc) atomicOr(&S->trunc, 1);
}
template <typename T, bool BG = false>
__global__ __launch_bounds__(kBlock) void k_emit_rows(const T* __restrict__ in, int64_t nx, Layout L, int64_t ny,
                                                      int64_t nrows, EmitOut o, const float* __restrict__ bg,
                                                      int bg_plane, const uint16_t* __restrict__ px) {
    k_emit_rows_body<T, BG>(hw_part(), in, nx, L, ny, nrows, o, bg, bg_plane, px);
}

hipError_t launch_emit(const LaunchCtx& lc, const Geom& g, const Layout& L, const void* in, roix_dtype dt,
                       const roix_fused_out* out, const BgRef* bg) {
    EmitOut o;
    o.rows = out->d_rows;
    o.rows_cap = out->d_rows ? (uint64_t)out->rows_cap : 0;
    o.stream = (uint8_t*)out->d_stream;
    o.stream_cap = out->d_stream ? (uint64_t)out->stream_cap_bytes : 0;
    o.outl = out->d_outliers;
    o.outl_cap = out->d_outliers ? (uint64_t)out->outliers_cap : 0;
    o.nvox = L.nvals ? L.nvals : g.N;
    const dim3 block(kBlock);
    const dim3 grid_rows_t(grid_rows(g.nrows, kBlock, lc.grid_stream));
    // a wave per chunk of kEmitChunk codes, at most one code per voxel: a
    // small volume launches only the waves its chunks can use
    const dim3 grid_waves(grid_rows((int64_t)((g.N + kEmitChunk - 1) / kEmitChunk), kBlock / kWave, lc.grid_emit));
    timer_begin(lc.timer, ST_EMIT, lc.stream);
    launch_k<kBlock, k_emit_index_body>(lc, k_emit_index, grid_rows_t, block, 0, L, g.nx, g.nrows);
    // the lean kernel queues the chunks it leaves to the general kernel
    if (dt == ROIX_F32) {
        // the 16-bit proxy (proxy element = voxel when rows are whole 64-voxel words)
        const uint16_t* px = (L.fine_slots && g.W * 64 == g.nx) ? reinterpret_cast<const uint16_t*>(L.proxy) : nullptr;
        // with a background the kernels that read voxel values read M
        const float* vals = bg ? bg->work : (const float*)in;
        launch_k<kBlock, k_emit_codes_f32_body>(lc, k_emit_codes_f32, grid_waves, block, 0, (const float*)in, vals, g.nx,
                                                L, o, px);
        if (bg) {
            hipError_t e = launch_background_if(lc, (const float*)in, *bg, g, L.S, 2);
            if (e != hipSuccess) return e;
        }
        launch_k<kBlock, k_emit_codes_general_body<float>>(lc, k_emit_codes_general<float>, grid_waves, block, 0, vals, g.nx, L, o);
    } else {
        launch_k<kBlock, k_emit_codes_body<uint16_t>>(lc, k_emit_codes<uint16_t>, grid_waves, block, 0, (const uint16_t*)in, g.nx, L, o, 0);
        launch_k<kBlock, k_emit_codes_general_body<uint16_t>>(lc, k_emit_codes_general<uint16_t>, grid_waves, block, 0, (const uint16_t*)in, g.nx,
                           L, o);
    }
    timer_end(lc.timer, ST_EMIT, lc.stream);
    hipError_t e = launch_scan_u64(lc, L.row_outl, L.row_outl, g.nrows, &L.S->n_outliers, L.scan_tmp);
    if (e != hipSuccess) return e;
    timer_begin(lc.timer, ST_EMIT_ROWS, lc.stream);
    // the 16-bit proxy when the layout holds one with element = voxel (the
    // kernel uses it only if the call took the one-pass flow)
    const uint16_t* px16 =
        (dt == ROIX_F32 && L.fine_slots && g.W * 64 == g.nx) ? reinterpret_cast<const uint16_t*>(L.proxy) : nullptr;
    if (dt == ROIX_F32 && bg) {
        launch_k<kBlock, k_emit_rows_body<float, true>>(lc, k_emit_rows<float, true>, grid_rows_t, block, 0, (const float*)in, g.nx, L,
                           g.ny, g.nrows, o, bg->bg, bg->plane ? 1 : 0, px16);
    } else if (dt == ROIX_F32) {
        launch_k<kBlock, k_emit_rows_body<float, false>>(lc, k_emit_rows<float, false>, grid_rows_t, block, 0, (const float*)in, g.nx, L,
                           g.ny, g.nrows, o, (const float*)nullptr, 0, px16);
    } else {
        launch_k<kBlock, k_emit_rows_body<uint16_t, false>>(lc, k_emit_rows<uint16_t, false>, grid_rows_t, block, 0, (const uint16_t*)in, g.nx,
                           L, g.ny, g.nrows, o, (const float*)nullptr, 0, (const uint16_t*)nullptr);
    }
    timer_end(lc.timer, ST_EMIT_ROWS, lc.stream);
    return hipGetLastError();
}

// --------------------------------------------------------------- finalize

__device__ __forceinline__ void k_finalize_body(const VPart vp, const DevState* S, roix_quant_info* qi, roix_seg_info* si, roix_extract_info* ei,
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
            for (int k = 0; k < 3; ++k) si->thresholds[k] = qbad ? -1 : S->thr_t[k];
            si->n_classes = qbad ? 0 : S->n_classes;
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
__global__ __launch_bounds__(1024) void k_finalize(const DevState* S, roix_quant_info* qi, roix_seg_info* si, roix_extract_info* ei,
                           int fused_q) {
    k_finalize_body(hw_part(), S, qi, si, ei, fused_q);
}

hipError_t launch_finalize(const LaunchCtx& lc, DevState* S, roix_quant_info* qi, roix_seg_info* si,
                           roix_extract_info* ei, bool fused_q) {
    timer_begin(lc.timer, ST_FINALIZE, lc.stream);
    launch_k<1024, k_finalize_body>(lc, k_finalize, dim3(1), dim3(256), 0, (const DevState*)S, qi, si, ei, fused_q ? 1 : 0);
    timer_end(lc.timer, ST_FINALIZE, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
