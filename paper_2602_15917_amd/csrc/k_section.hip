// k_section.hip - the normalised 8-bit pixel section of an extraction
// (Sec. 4.1.2, Eq. 1): for every span voxel, in the order of the code
// stream, the level floor(256 (q - qmin) / K) of its quantisation code.
//
// The section is derived from the stored code stream, not from the volume:
// a stored code u = q - qmin gives the level at once, so the pass reads the
// stream (1, 2 or 4 bytes per code) and writes one byte per code, flat and
// coalesced, with no row table in the way.  Only an escaped code (an
// outlier, whose q is not stored) needs its voxel: a binary search over the
// rows' first codes gives its row and the voxel is requantised.  Escapes are
// rare, so this costs nothing on the common path.
#include "common.h"

namespace roix {

constexpr int kSecCodes = 16;  // codes per thread and step: one 16-byte store

// The call's status and code count, checked once before the pass.
__global__ void k_section_check(const roix_quant_info* __restrict__ qi, const roix_extract_info* __restrict__ ei,
                                int64_t rows_cap, int64_t stream_cap, int64_t out_cap, roix_section_info* info) {
    int32_t st = qi->status != ROIX_OK ? qi->status : ei->status;
    const uint64_t n = ei->n_codes;
    if (st == ROIX_OK) {
        const int wb = qi->width_bits;
        if (wb != 8 && wb != 16 && wb != 32) st = ROIX_EINVAL;
        else if (ei->n_rows > (uint64_t)rows_cap || n * (uint64_t)(wb / 8) > (uint64_t)stream_cap)
            st = ROIX_EINVAL;  // the stream or the row table was not written whole
        else if (n > (uint64_t)out_cap)
            st = ROIX_ETRUNC;
    }
    info->status = st;
    info->pad = 0;
    info->n_codes = n;
}

struct SecParams {
    uint32_t K, mlo, mhi, esc;
    float binscale, r;
    int32_t qmin;
    bool fast;
};

__device__ __forceinline__ SecParams sec_params(const roix_quant_info* __restrict__ qi) {
    SecParams p;
    p.K = (uint32_t)qi->K;
    // ceil(2^40 / K) for the exact multiply-high division (K <= 65536)
    const uint64_t M = ((1ull << 40) + (uint64_t)p.K - 1) / (uint64_t)p.K;
    p.mlo = (uint32_t)M;
    p.mhi = (uint32_t)(M >> 32);
    p.fast = p.K <= 65536u;
    p.binscale = (float)(256.0 / (double)p.K);
    p.esc = qi->esc;
    p.r = qi->r;
    p.qmin = qi->qmin;
    return p;
}

__device__ __forceinline__ uint32_t sec_level(uint32_t u, const SecParams& p) {
    return p.fast ? bin_fast(u, p.mlo, p.mhi) : bin_slow(u, p.K, p.binscale);
}

// The level of the escaped code c: its row is the last one whose first code
// is at or before c; the voxel is requantised with the call's quantiser.
template <typename T>
__device__ uint32_t sec_escape(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
                               const roix_row* __restrict__ rows, uint64_t nr, uint64_t c, const SecParams& p,
                               roix_section_info* info) {
    if (nr == 0) {
        atomicCAS(&info->status, (int32_t)ROIX_OK, (int32_t)ROIX_EINVAL);  // a row table that does not cover the stream
        return 0;
    }
    uint64_t lo = 0, hi = nr;  // rows[lo].code_off <= c < rows[hi].code_off
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (rows[mid].code_off <= c) lo = mid;
        else hi = mid;
    }
    const roix_row r = rows[lo];
    const uint64_t dx = c - r.code_off;
    if (r.code_off > c || r.z >= (uint64_t)nz || r.y >= (uint64_t)ny || r.xe > (uint64_t)nx ||
        dx >= (uint64_t)(r.xe - r.xs)) {
        atomicCAS(&info->status, (int32_t)ROIX_OK, (int32_t)ROIX_EINVAL);  // a row table that does not cover the stream
        return 0;
    }
    const float x = (float)in[((uint64_t)r.z * (uint64_t)ny + r.y) * (uint64_t)nx + r.xs + dx];
    const uint32_t lv = sec_level((uint32_t)(qcode(x, p.r) - p.qmin), p);
    return lv > 255u ? 255u : lv;  // (only a volume other than the extracted one gives a code outside 0..K-1)
}

// code i of a 16-byte word group of B-byte codes
template <int B>
__device__ __forceinline__ uint32_t code_at(const uint4 (&w)[B], int i) {
    const uint32_t word = i * B / 4;
    const uint32_t v = (word & 3) == 0 ? w[word >> 2].x : (word & 3) == 1 ? w[word >> 2].y
                     : (word & 3) == 2 ? w[word >> 2].z : w[word >> 2].w;
    if (B == 4) return v;
    if (B == 2) return (v >> (16 * (i & 1))) & 0xFFFFu;
    return (v >> (8 * (i & 3))) & 0xFFu;
}

template <typename T, int B>
__device__ void section_pass(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
                             const roix_row* __restrict__ rows, uint64_t nr, const uint8_t* __restrict__ stream,
                             uint64_t n, const SecParams& p, uint8_t* __restrict__ out, roix_section_info* info) {
    const uint64_t ng = n / kSecCodes;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += stride) {
        uint4 w[B];
        const uint4* src = reinterpret_cast<const uint4*>(stream + g * (kSecCodes * B));
#pragma unroll
        for (int k = 0; k < B; ++k) w[k] = ld_stream(src + k);
        uint32_t lv[kSecCodes];
        bool any_esc = false;
#pragma unroll
        for (int i = 0; i < kSecCodes; ++i) {
            const uint32_t u = code_at<B>(w, i);
            any_esc |= u == p.esc;
            lv[i] = u == p.esc ? 0u : sec_level(u, p);
        }
        if (any_esc) {
            for (int i = 0; i < kSecCodes; ++i)
                if (code_at<B>(w, i) == p.esc) lv[i] = sec_escape(in, nx, ny, nz, rows, nr, g * kSecCodes + i, p, info);
        }
        uint4 o;
        o.x = lv[0] | lv[1] << 8 | lv[2] << 16 | lv[3] << 24;
        o.y = lv[4] | lv[5] << 8 | lv[6] << 16 | lv[7] << 24;
        o.z = lv[8] | lv[9] << 8 | lv[10] << 16 | lv[11] << 24;
        o.w = lv[12] | lv[13] << 8 | lv[14] << 16 | lv[15] << 24;
        v4u32_t t;
        t.x = o.x;
        t.y = o.y;
        t.z = o.z;
        t.w = o.w;
        __builtin_nontemporal_store(t, reinterpret_cast<v4u32_t*>(out + g * kSecCodes));
    }
    // the last n mod 16 codes, one thread each
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t c = ng * kSecCodes + t;
    if (c < n) {
        uint32_t u;
        if (B == 1) u = stream[c];
        else if (B == 2) u = reinterpret_cast<const uint16_t*>(stream)[c];
        else u = reinterpret_cast<const uint32_t*>(stream)[c];
        out[c] = (uint8_t)(u == p.esc ? sec_escape(in, nx, ny, nz, rows, nr, c, p, info) : sec_level(u, p));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_section(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
                                                    const roix_quant_info* __restrict__ qi,
                                                    const roix_extract_info* __restrict__ ei,
                                                    const roix_row* __restrict__ rows,
                                                    const uint8_t* __restrict__ stream, uint8_t* __restrict__ out,
                                                    roix_section_info* info) {
    if (info->status != ROIX_OK) return;
    const SecParams p = sec_params(qi);
    const uint64_t n = ei->n_codes, nr = ei->n_rows;
    const int wb = qi->width_bits;
    if (wb == 8) section_pass<T, 1>(in, nx, ny, nz, rows, nr, stream, n, p, out, info);
    else if (wb == 16) section_pass<T, 2>(in, nx, ny, nz, rows, nr, stream, n, p, out, info);
    else section_pass<T, 4>(in, nx, ny, nz, rows, nr, stream, n, p, out, info);
}

hipError_t launch_section(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g,
                          const roix_fused_out* o, uint8_t* out, int64_t out_cap, roix_section_info* info) {
    timer_begin(lc.timer, ST_SECTION, lc.stream);
    hipLaunchKernelGGL(k_section_check, dim3(1), dim3(1), 0, lc.stream, o->d_qinfo, o->d_einfo, o->rows_cap,
                       o->stream_cap_bytes, out_cap, info);
    const dim3 grid(lc.grid_stream), block(kBlock);
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_section<float>, grid, block, 0, lc.stream, (const float*)in, g.nx, g.ny, g.nz,
                           o->d_qinfo, o->d_einfo, o->d_rows, (const uint8_t*)o->d_stream, out, info);
    else
        hipLaunchKernelGGL(k_section<uint16_t>, grid, block, 0, lc.stream, (const uint16_t*)in, g.nx, g.ny, g.nz,
                           o->d_qinfo, o->d_einfo, o->d_rows, (const uint8_t*)o->d_stream, out, info);
    timer_end(lc.timer, ST_SECTION, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
