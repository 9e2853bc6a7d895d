// k_decode.hip - the reverse process: a float32 volume from the row table,
// the packed code stream and the outliers.
//
// Every voxel of the output is written exactly once.  An index kernel checks
// the table (rows inside the volume, xs < xe, strictly increasing raster
// order, codes inside the stream, outlier offsets that never decrease) and
// writes a 32-byte descriptor per volume row: its span, first code, first
// outlier and the number of escapes the offsets imply (an empty span for a
// row without an entry).  Then a wave takes 64 volume rows at a time, one
// descriptor per lane, and walks them in units of 512 voxels, the code
// loads of the next unit in flight while the current one is written:
// background outside the span, (u + qmin) * w inside it, the k-th escape of
// the row taking outlier outlier_off + k (a wave prefix count, skipped when
// a step has no escape).  At the end of a row the wave checks that it met as
// many escapes as the descriptor says.
#include "common.h"

namespace roix {

struct DecodeArgs {
    const roix_row* rows;
    uint64_t rows_cap;
    const uint8_t* stream;
    uint64_t stream_cap;  // bytes
    const float* outl;
    uint64_t outl_cap;
    const roix_quant_info* qi;
    const roix_extract_info* ei;
    int64_t nx, ny, nz;
    float background;
    float* out;
    uint4* desc;    // 2 * ny * nz: per volume row {xs, xe, code_off lo, hi}, {outl lo, hi, escapes lo, hi}
    DevState* S;
};

// counts of the table, each bounded by its buffer's capacity (a count above
// it is an error found by k_decode_check)
__device__ __forceinline__ uint64_t dec_rows(const DecodeArgs& a) {
    const uint64_t n = a.ei->n_rows;
    return n < a.rows_cap ? n : a.rows_cap;
}

__global__ void k_decode_check(DecodeArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState* S = a.S;
    S->status = 0;
    const roix_quant_info* q = a.qi;
    const roix_extract_info* e = a.ei;
    const int wb = q->width_bits;
    bool ok = q->status == 0 && e->status == 0 && (wb == 8 || wb == 16 || wb == 32);
    ok = ok && e->n_rows <= a.rows_cap && e->n_outliers <= a.outl_cap;
    ok = ok && wb != 0 && e->n_codes <= a.stream_cap / (uint64_t)(wb / 8);
    ok = ok && q->esc == (wb == 32 ? 0xFFFFFFFFu : ((1u << wb) - 1u));
    ok = ok && e->n_rows <= (uint64_t)(a.ny * a.nz);
    if (!ok) S->status = ROIX_EINVAL;
}

__global__ __launch_bounds__(kBlock) void k_decode_clear(DecodeArgs a, int64_t nrows) {
    const int64_t n = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += n) {
        a.desc[2 * r] = make_uint4(0u, 0u, 0u, 0u);
        a.desc[2 * r + 1] = make_uint4(0u, 0u, 0u, 0u);
    }
}

__global__ __launch_bounds__(kBlock) void k_decode_index(DecodeArgs a) {
    const uint64_t n = dec_rows(a);
    // codes a row may reference: the count, bounded by what the stream holds
    // (a larger count is an error found by k_decode_check), so that no
    // described row reads past the stream
    const uint64_t cb = (uint64_t)(a.qi->width_bits / 8);
    const uint64_t cap_codes = (cb == 1 || cb == 2 || cb == 4) ? a.stream_cap / cb : 0ull;
    const uint64_t n_codes = a.ei->n_codes < cap_codes ? a.ei->n_codes : cap_codes;
    const uint64_t n_outl = a.ei->n_outliers;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nthreads) {
        const roix_row e = a.rows[i];
        bool ok = (int64_t)e.z < a.nz && (int64_t)e.y < a.ny && e.xs < e.xe && (int64_t)e.xe <= a.nx;
        ok = ok && e.code_off <= n_codes && (uint64_t)(e.xe - e.xs) <= n_codes - e.code_off;
        const uint64_t rid = (uint64_t)e.z * (uint64_t)a.ny + e.y;
        if (i == 0) {
            ok = ok && e.outlier_off == 0ull;
        } else {
            const roix_row p = a.rows[i - 1];
            ok = ok && ((uint64_t)p.z * (uint64_t)a.ny + p.y) < rid;
        }
        const uint64_t onext = i + 1 < n ? a.rows[i + 1].outlier_off : n_outl;
        ok = ok && onext >= e.outlier_off;
        if (ok) {
            const uint64_t ne = onext - e.outlier_off;
            a.desc[2 * rid] = make_uint4(e.xs, e.xe, (uint32_t)e.code_off, (uint32_t)(e.code_off >> 32));
            a.desc[2 * rid + 1] =
                make_uint4((uint32_t)e.outlier_off, (uint32_t)(e.outlier_off >> 32), (uint32_t)ne, (uint32_t)(ne >> 32));
        } else {
            bad = true;
        }
    }
    if (bad) fail(a.S, ROIX_EINVAL);
}

template <int B>
__device__ __forceinline__ uint32_t code1(const uint8_t* __restrict__ s, uint64_t c) {
    if constexpr (B == 4)
        return reinterpret_cast<const uint32_t*>(s)[c];
    else if constexpr (B == 2)
        return reinterpret_cast<const uint16_t*>(s)[c];
    else
        return s[c];
}

// Bytes a whole four-code load at code c touches, counted from byte 0.
template <int B>
__device__ __forceinline__ uint64_t codes4_end(uint64_t c) {
    if constexpr (B == 4)
        return 4 * c + 16;
    else if constexpr (B == 2)
        return ((2 * c) & ~3ull) + 12;
    else
        return (c & ~3ull) + 8;
}

// The dwords of a four-code window at code c (B = 4: the codes themselves).
template <int B>
__device__ __forceinline__ void window_load(const uint8_t* __restrict__ s, uint64_t c, uint32_t (&d)[4]) {
    if constexpr (B == 4) {
        const v4u32_t q = *(reinterpret_cast<const v4u32_t*>(s + 4 * c));
        d[0] = q.x;
        d[1] = q.y;
        d[2] = q.z;
        d[3] = q.w;
    } else if constexpr (B == 2) {
        const v3u32_t q = *(reinterpret_cast<const v3u32_t*>(s + ((2 * c) & ~3ull)));
        d[0] = q.x;
        d[1] = q.y;
        d[2] = q.z;
        d[3] = 0u;
    } else {
        const v2u32_t q = *(reinterpret_cast<const v2u32_t*>(s + (c & ~3ull)));
        d[0] = q.x;
        d[1] = q.y;
        d[2] = d[3] = 0u;
    }
}

template <int B>
__device__ __forceinline__ void window_codes(const uint32_t (&d)[4], uint64_t c, uint32_t (&u)[4]) {
    if constexpr (B == 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = d[j];
    } else {
        const uint32_t sh = (uint32_t)((c * B) & 3ull) * 8u;
        const uint32_t w0 = __builtin_amdgcn_alignbit(d[1], d[0], sh), w1 = __builtin_amdgcn_alignbit(d[2], d[1], sh);
        if constexpr (B == 2) {
            u[0] = w0 & 0xFFFFu;
            u[1] = w0 >> 16;
            u[2] = w1 & 0xFFFFu;
            u[3] = w1 >> 16;
        } else {
            u[0] = w0 & 0xFFu;
            u[1] = (w0 >> 8) & 0xFFu;
            u[2] = (w0 >> 16) & 0xFFu;
            u[3] = w0 >> 24;
        }
    }
}

constexpr int kDecSteps = 2;                             // 256-voxel steps per unit
constexpr int64_t kDecUnit = (int64_t)kDecSteps * 4 * kWave;  // voxels per unit

// Descriptor of row j of the wave's group (lane j holds it), uniform.
struct RowDesc {
    uint32_t xs, xe;
    uint64_t coff, ooff, nesc;
};
__device__ __forceinline__ RowDesc row_desc(const uint4& d0, const uint4& d1, int j) {
    RowDesc r;
    r.xs = __builtin_amdgcn_readlane(d0.x, j);
    r.xe = __builtin_amdgcn_readlane(d0.y, j);
    r.coff = ((uint64_t)__builtin_amdgcn_readlane(d0.w, j) << 32) | __builtin_amdgcn_readlane(d0.z, j);
    r.ooff = ((uint64_t)__builtin_amdgcn_readlane(d1.y, j) << 32) | __builtin_amdgcn_readlane(d1.x, j);
    r.nesc = ((uint64_t)__builtin_amdgcn_readlane(d1.w, j) << 32) | __builtin_amdgcn_readlane(d1.z, j);
    return r;
}

// The code windows of one unit (voxels x0 .. of a row): a lane whose four
// voxels overlap the span loads the window of codes c = coff + x - xs; one
// that cannot (the window would start before code 0 or end past the stream)
// is redone code by code after the unit's stores.  Every other lane loads
// the stream's first window (one cached line for all of them), so that no
// load sits under a branch and the wait counts stay exact.  Coordinates are
// 32-bit (nx < 2^31).
template <int B>
__device__ __forceinline__ void unit_load(const DecodeArgs& a, const RowDesc& rd, int32_t x0,
                                          uint32_t (&raw)[kDecSteps][4]) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int s = 0; s < kDecSteps; ++s) {
        const int32_t dx = x0 + s * 4 * kWave + 4 * lane - (int32_t)rd.xs;  // voxel x - xs
        const int64_t c = (int64_t)rd.coff + dx;
        const bool over = dx + 4 > 0 && dx < (int32_t)(rd.xe - rd.xs);
        const bool ok = over && c >= 0 && codes4_end<B>((uint64_t)c) <= a.stream_cap;
        window_load<B>(a.stream, ok ? (uint64_t)c : 0ull, raw[s]);
    }
}

// Writes one unit from its loaded windows; escapes and lanes without a
// window are left to unit_fix (returned in fix, uniform).  No loads.
template <int B>
__device__ __forceinline__ bool unit_write(const DecodeArgs& a, const RowDesc& rd, int32_t x0, float* dst,
                                           const uint32_t (&raw)[kDecSteps][4], bool vec_out, int32_t qmin, float w,
                                           uint32_t esc, float bg) {
    const int lane = threadIdx.x % kWave;
    const int32_t nx = (int32_t)a.nx;
    const uint32_t len = rd.xe - rd.xs;
    bool fix = false;
#pragma unroll
    for (int s = 0; s < kDecSteps; ++s) {
        const int32_t xs0 = x0 + s * 4 * kWave;
        if (xs0 >= nx) break;  // uniform
        const int32_t x = xs0 + 4 * lane;
        float v[4];
        const bool any_span = xs0 < (int32_t)rd.xe && xs0 + 4 * kWave > (int32_t)rd.xs;  // uniform
        if (!any_span) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = bg;
        } else {
            const int32_t dx = x - (int32_t)rd.xs;
            const int64_t c = (int64_t)rd.coff + dx;
            const bool over = dx + 4 > 0 && dx < (int32_t)len;
            const bool ok = c >= 0 && codes4_end<B>((uint64_t)c) <= a.stream_cap;
            uint32_t cu[4];
            window_codes<B>(raw[s], (uint64_t)c, cu);
            bool e = over && !ok;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = (uint32_t)(dx + q) < len;
                e = e || (in && cu[q] == esc);
                v[q] = in ? (float)(int32_t)(cu[q] + (uint32_t)qmin) * w : bg;
            }
            fix = fix || __ballot(e) != 0ull;
        }
        if (vec_out && xs0 + 4 * kWave <= nx) {  // uniform: every lane's four voxels exist
            v4u32_t t;
            t.x = __float_as_uint(v[0]);
            t.y = __float_as_uint(v[1]);
            t.z = __float_as_uint(v[2]);
            t.w = __float_as_uint(v[3]);
            __builtin_nontemporal_store(t, reinterpret_cast<v4u32_t*>(dst + x));
        } else if (vec_out) {
            if (x < nx) {
                v4u32_t t;
                t.x = __float_as_uint(v[0]);
                t.y = __float_as_uint(v[1]);
                t.z = __float_as_uint(v[2]);
                t.w = __float_as_uint(v[3]);
                __builtin_nontemporal_store(t, reinterpret_cast<v4u32_t*>(dst + x));
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (x + q < nx) dst[x + q] = v[q];
        }
    }
    return fix;
}

// Rare: the unit's span voxels again, code by code, in order of x, storing
// the outlier values of escapes (and every code of a lane without a window).
// Advances k by the unit's escapes.
template <int B>
__device__ __forceinline__ void unit_fix(const DecodeArgs& a, const RowDesc& rd, int32_t x0, float* dst,
                                         int32_t qmin, float w, uint32_t esc, uint64_t n_out, uint64_t& k, bool& bad) {
    const int lane = threadIdx.x % kWave;
    const int32_t nx = (int32_t)a.nx;
    const uint32_t len = rd.xe - rd.xs;
    for (int s = 0; s < kDecSteps; ++s) {
        const int32_t xs0 = x0 + s * 4 * kWave;
        if (xs0 >= nx) break;
        if (!(xs0 < (int32_t)rd.xe && xs0 + 4 * kWave > (int32_t)rd.xs)) continue;
        const int32_t dx = xs0 + 4 * lane - (int32_t)rd.xs;
        uint32_t cu[4];
        uint32_t em = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool in = (uint32_t)(dx + q) < len;
            cu[q] = in ? code1<B>(a.stream, rd.coff + (uint64_t)(dx + q)) : 0u;
            em |= (in && cu[q] == esc) ? (1u << q) : 0u;
        }
        const uint32_t cnt = (uint32_t)__popc(em);
        uint32_t incl = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        uint64_t at = k + (incl - cnt);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!((uint32_t)(dx + q) < len)) continue;
            float v;
            if ((em >> q) & 1u) {
                if (at < n_out) {
                    v = a.outl[at];
                } else {
                    v = 0.0f;
                    bad = true;
                }
                ++at;
            } else {
                v = (float)(int32_t)(cu[q] + (uint32_t)qmin) * w;
            }
            dst[rd.xs + dx + q] = v;
        }
        k += (uint64_t)__shfl(incl, kWave - 1);
    }
}

template <int B>
__device__ __forceinline__ void decode_rows(const DecodeArgs& a, bool vec_out) {
    const int lane = threadIdx.x % kWave;
    const int64_t nrows = a.ny * a.nz;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    const uint64_t n_out = a.ei->n_outliers < a.outl_cap ? a.ei->n_outliers : a.outl_cap;
    const int32_t qmin = a.qi->qmin;
    const float w = a.qi->w;
    const uint32_t esc = a.qi->esc;
    const float bg = a.background;
    const int32_t nx = (int32_t)a.nx;
    bool bad = false;
    // Every whole-window load reads inside the stream (c >= 0 and the
    // window's end within the capacity, else the window at code 0); a stream
    // too small for one window at code 0 is decoded code by code only.
    const bool wl = codes4_end<B>(0) <= a.stream_cap;
    for (int64_t g0 = wave * kWave; g0 < nrows; g0 += nwaves * kWave) {
        const int64_t rl = g0 + lane;
        uint4 d0 = make_uint4(0u, 0u, 0u, 0u), d1 = make_uint4(0u, 0u, 0u, 0u);
        if (rl < nrows) {
            d0 = a.desc[2 * rl];
            d1 = a.desc[2 * rl + 1];
        }
        const int nr = (int)(nrows - g0 < kWave ? nrows - g0 : kWave);
        uint64_t k = 0;  // outlier index of the row's next escape
        // one unit (row j, voxels x0 ..): the write, the rare fix-up, the row-end check
        auto run = [&](int j, int32_t x0, const uint32_t(&raw)[kDecSteps][4], bool loaded) {
            const RowDesc rd = row_desc(d0, d1, j);
            if (x0 == 0) k = rd.ooff;
            float* dst = a.out + (g0 + j) * (int64_t)nx;
            // without windows the write only places the background and the
            // fix-up writes every span voxel
            const bool fix = unit_write<B>(a, rd, x0, dst, raw, vec_out, qmin, w, esc, bg) || !loaded;
            if (fix) unit_fix<B>(a, rd, x0, dst, qmin, w, esc, n_out, k, bad);
            if (x0 + kDecUnit >= nx && rd.xe > rd.xs && k - rd.ooff != rd.nesc) bad = true;
        };
        // unit cursor: row j, first voxel x0; next() steps to the following unit
        auto next = [&](int& j, int32_t& x0) {
            x0 += (int32_t)kDecUnit;
            if (x0 >= nx) {
                x0 = 0;
                ++j;
            }
        };
        if (wl) {  // uniform
            // ping-pong: the next unit's windows are in flight while this one
            // is written; past the last row the loads repeat row 0 (harmless)
            auto load = [&](int j, int32_t x0, uint32_t(&raw)[kDecSteps][4]) {
                const bool past = j >= nr;
                unit_load<B>(a, row_desc(d0, d1, past ? 0 : j), past ? 0 : x0, raw);
            };
            uint32_t ra[kDecSteps][4], rb[kDecSteps][4];
            int ja = 0, jb = 0;
            int32_t xa = 0, xb = 0;
            load(ja, xa, ra);
            while (ja < nr) {
                jb = ja;
                xb = xa;
                next(jb, xb);
                load(jb, xb, rb);
                run(ja, xa, ra, true);
                ja = jb;
                xa = xb;
                next(ja, xa);
                load(ja, xa, ra);
                if (jb < nr) run(jb, xb, rb, true);
            }
        } else {
            uint32_t rz[kDecSteps][4] = {};
            for (int j = 0; j < nr; ++j)
                for (int32_t x0 = 0; x0 < nx; x0 += (int32_t)kDecUnit) run(j, x0, rz, false);
        }
    }
    if (bad) fail(a.S, ROIX_EINVAL);
}

// One kernel per code width (the width is device data: the two kernels of
// the other widths return at once), so that each keeps its own registers.
// vec_out: rows start 16-byte aligned (nx % 4 == 0 and an aligned output).
template <int B>
__global__ __launch_bounds__(kBlock) void k_decode_rows(DecodeArgs a, int vec_out) {
    if (a.qi->width_bits != 8 * B) return;
    decode_rows<B>(a, vec_out != 0);
}

__global__ void k_decode_finish(DecodeArgs a, roix_decode_info* d) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    d->status = a.S->status;
    d->pad = 0;
    d->n_rows = a.ei->n_rows;
    d->n_codes = a.ei->n_codes;
    d->n_outliers = a.ei->n_outliers;
}

hipError_t launch_decode(const LaunchCtx& lc, const roix_row* rows, uint64_t rows_cap, const void* stream,
                         uint64_t stream_cap, const float* outl, uint64_t outl_cap, const roix_quant_info* qi,
                         const roix_extract_info* ei, const Geom& g, float background, float* out, DevState* S,
                         uint4* desc, roix_decode_info* dinfo) {
    DecodeArgs a;
    a.rows = rows;
    a.rows_cap = rows ? rows_cap : 0;
    a.stream = (const uint8_t*)stream;
    a.stream_cap = stream ? stream_cap : 0;
    a.outl = outl;
    a.outl_cap = outl ? outl_cap : 0;
    a.qi = qi;
    a.ei = ei;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.background = background;
    a.out = out;
    a.desc = desc;
    a.S = S;
    const int vec_out = (g.nx % 4 == 0 && (uintptr_t)out % 16 == 0) ? 1 : 0;
    int64_t gr = (g.nrows + kBlock - 1) / kBlock;
    const int grid_r = (int)(gr < lc.grid_stream ? (gr < 1 ? 1 : gr) : lc.grid_stream);
    timer_begin(lc.timer, ST_DECODE_INDEX, lc.stream);
    hipLaunchKernelGGL(k_decode_check, dim3(1), dim3(64), 0, lc.stream, a);
    hipLaunchKernelGGL(k_decode_clear, dim3(grid_r), dim3(kBlock), 0, lc.stream, a, g.nrows);
    hipLaunchKernelGGL(k_decode_index, dim3(grid_r), dim3(kBlock), 0, lc.stream, a);
    timer_end(lc.timer, ST_DECODE_INDEX, lc.stream);
    timer_begin(lc.timer, ST_DECODE, lc.stream);
    hipLaunchKernelGGL(k_decode_rows<2>, dim3(lc.grid_stream), dim3(kBlock), 0, lc.stream, a, vec_out);
    hipLaunchKernelGGL(k_decode_rows<1>, dim3(lc.grid_stream), dim3(kBlock), 0, lc.stream, a, vec_out);
    hipLaunchKernelGGL(k_decode_rows<4>, dim3(lc.grid_stream), dim3(kBlock), 0, lc.stream, a, vec_out);
    timer_end(lc.timer, ST_DECODE, lc.stream);
    hipLaunchKernelGGL(k_decode_finish, dim3(1), dim3(64), 0, lc.stream, a, dinfo);
    return hipGetLastError();
}

}  // namespace roix
