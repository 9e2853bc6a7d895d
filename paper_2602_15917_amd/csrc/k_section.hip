// k_section.hip - the normalised 8-bit pixel section of an extraction
// (Sec. 4.1.2, Eq. 1): for every span voxel, in the order of the code
// stream, the level floor(256 (q - qmin) / K) of its quantisation code.
//
// The section is derived from the stored code stream, not from the volume:
// a stored code u = q - qmin gives the level at once, so the pass reads the
// stream (1, 2 or 4 bytes per code) and writes one byte per code, flat and
// coalesced, with no row table in the way.  Only an escaped code (an
// outlier, whose q is not stored) needs its voxel: a binary search over the
// rows' first codes gives its row and the voxel is requantised.  That search
// is a chain of dependent loads which would stall its whole wave, so the
// streaming pass only lists the escaped codes (in the context's arena, each
// workgroup in a part of its own, counted in LDS) and a second kernel
// resolves them, one thread each.
#include "common.h"

namespace roix {

// The call's status and code count, checked once before the pass.
// The escape list: workgroup w lists its escaped codes in
// list[w * per .. (w + 1) * per) and their number in count[w] (which may
// exceed per: the rest were resolved in place).
struct SecEsc {
    unsigned long long* count;  // ngroups entries
    unsigned long long* list;
    unsigned long long per;
    uint32_t ngroups;
};

__global__ void k_section_check(const roix_quant_info* __restrict__ qi, const roix_extract_info* __restrict__ ei,
                                int64_t rows_cap, int64_t stream_cap, int64_t out_cap, roix_section_info* info,
                                SecEsc esc) {
    for (uint32_t w = threadIdx.x; w < esc.ngroups; w += blockDim.x) esc.count[w] = 0ull;
    if (threadIdx.x != 0) return;
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
    uint32_t K, mlo, mhi, esc, a24, m24;
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
    bin24_params(p.K, p.a24, p.m24);
    p.binscale = (float)(256.0 / (double)p.K);
    p.esc = qi->esc;
    p.r = qi->r;
    p.qmin = qi->qmin;
    return p;
}

__device__ __forceinline__ uint32_t sec_level(uint32_t u, const SecParams& p) {
    return p.m24 ? bin24(u, p.a24, p.m24) : (p.fast ? bin_fast(u, p.mlo, p.mhi) : bin_slow(u, p.K, p.binscale));
}
// the same with the form fixed at compile time (DIV 2: 24-bit, 1: 32-bit, 0: float estimate)
template <int DIV>
__device__ __forceinline__ uint32_t sec_level_d(uint32_t u, const SecParams& p) {
    return DIV == 2 ? bin24(u, p.a24, p.m24) : (DIV == 1 ? bin_fast(u, p.mlo, p.mhi) : bin_slow(u, p.K, p.binscale));
}

// The level of the escaped code c: its row is the last one whose first code
// is at or before c; the voxel is requantised with the call's quantiser.
template <typename T>
__device__ __attribute__((noinline)) uint32_t sec_escape(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
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

constexpr int kSecCodes = 16;  // codes per unit of work: B 16-byte loads, one 16-byte store

// code i of the B 16-byte loads of a unit
template <int B>
__device__ __forceinline__ uint32_t code_at(const uint4 (&w)[B], int i) {
    const int word = i * B / 4;
    const uint4& q = w[word >> 2];
    const uint32_t v = (word & 3) == 0 ? q.x : (word & 3) == 1 ? q.y : (word & 3) == 2 ? q.z : q.w;
    if (B == 4) return v;
    if (B == 2) return (v >> (16 * (i & 1))) & 0xFFFFu;
    return (v >> (8 * (i & 3))) & 0xFFu;
}

// The 16 levels of a unit, packed for one 16-byte store (escapes resolved).
// Every index into the codes is static (the escapes are found through a bit
// mask), so codes and levels stay in registers.
template <typename T, int B, int DIV>
__device__ __forceinline__ v4u32_t levels16(const uint4 (&w)[B], uint64_t c0, const T* __restrict__ in, int64_t nx,
                                            int64_t ny, int64_t nz, const roix_row* __restrict__ rows, uint64_t nr,
                                            const SecParams& p, roix_section_info* info, const SecEsc& esc,
                                            uint32_t* s_cnt) {
    uint32_t o[4] = {0u, 0u, 0u, 0u};
    uint32_t emask = 0;
#pragma unroll
    for (int i = 0; i < kSecCodes; ++i) {
        const uint32_t u = code_at<B>(w, i);
        emask |= (uint32_t)(u == p.esc) << i;
        o[i / 4] |= (u == p.esc ? 0u : sec_level_d<DIV>(u, p)) << (8 * (i & 3));
    }
    while (emask) {  // listed for the escape kernel (their level stays 0 here), or resolved in place
        const int i = __builtin_ctz(emask);
        emask &= emask - 1u;
        const uint32_t slot = atomicAdd(s_cnt, 1u);
        if (slot < esc.per) {
            esc.list[(unsigned long long)blockIdx.x * esc.per + slot] = c0 + (uint64_t)i;
            continue;
        }
        const uint32_t sh = 8u * (uint32_t)(i & 3);
        const uint32_t v = sec_escape(in, nx, ny, nz, rows, nr, c0 + (uint64_t)i, p, info) << sh;
        const int k = i >> 2;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (m == k) o[m] = (o[m] & ~(0xFFu << sh)) | v;
    }
    v4u32_t t;
    t.x = o[0];
    t.y = o[1];
    t.z = o[2];
    t.w = o[3];
    return t;
}

// Each thread takes units of 16 codes, kSecUnroll of them per step (a grid
// stride apart, so that each store instruction of a wave is one contiguous
// run and each load instruction one run with a stride of B 16-byte words),
// all loads of a step issued before any use (4 units; 2 of 32-bit codes,
// whose loads take twice the registers).
template <int B>
constexpr int sec_unroll() { return B == 4 ? 2 : 4; }

template <typename T, int B, int DIV>
__device__ void section_pass(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
                             const roix_row* __restrict__ rows, uint64_t nr, const uint8_t* __restrict__ stream,
                             uint64_t n, const SecParams& p, uint8_t* __restrict__ out, roix_section_info* info,
                             const SecEsc& esc, uint32_t* s_cnt) {
    const uint64_t nu = n / kSecCodes;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint4* src = reinterpret_cast<const uint4*>(stream);
    constexpr int kSecUnroll = sec_unroll<B>();
    for (uint64_t u0 = tid; u0 < nu; u0 += kSecUnroll * stride) {
        uint4 w[kSecUnroll][B];
#pragma unroll
        for (int k = 0; k < kSecUnroll; ++k) {
            const uint64_t u = u0 + k * stride;
            if (u < nu) {
#pragma unroll
                for (int j = 0; j < B; ++j) w[k][j] = ld_stream(src + u * B + j);
            }
        }
#pragma unroll
        for (int k = 0; k < kSecUnroll; ++k) {
            const uint64_t u = u0 + k * stride;
            if (u < nu) {
                const v4u32_t t = levels16<T, B, DIV>(w[k], u * kSecCodes, in, nx, ny, nz, rows, nr, p, info, esc, s_cnt);
                __builtin_nontemporal_store(t, reinterpret_cast<v4u32_t*>(out + u * kSecCodes));
            }
        }
    }
    // the last n mod 16 codes, one thread each
    const uint64_t c = nu * kSecCodes + tid;
    if (c < n) {
        uint32_t u;
        if (B == 1) u = stream[c];
        else if (B == 2) u = reinterpret_cast<const uint16_t*>(stream)[c];
        else u = reinterpret_cast<const uint32_t*>(stream)[c];
        out[c] = (uint8_t)(u == p.esc ? sec_escape(in, nx, ny, nz, rows, nr, c, p, info) : sec_level(u, p));
    }
}

// One kernel per code width, each returning at once unless the call's codes
// have its width: the width is device data, and a kernel of its own gives
// each width its own register budget (and so its own occupancy).
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_section(const T* __restrict__ in, int64_t nx, int64_t ny, int64_t nz,
                                                    const roix_quant_info* __restrict__ qi,
                                                    const roix_extract_info* __restrict__ ei,
                                                    const roix_row* __restrict__ rows,
                                                    const uint8_t* __restrict__ stream, uint8_t* __restrict__ out,
                                                    roix_section_info* info, SecEsc esc) {
    if (info->status != ROIX_OK || qi->width_bits != 8 * B) return;  // (uniform)
    __shared__ uint32_t s_cnt;  // this workgroup's listed escapes
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const SecParams p = sec_params(qi);
    if (p.m24)  // uniform
        section_pass<T, B, 2>(in, nx, ny, nz, rows, ei->n_rows, stream, ei->n_codes, p, out, info, esc, &s_cnt);
    else if (p.fast)
        section_pass<T, B, 1>(in, nx, ny, nz, rows, ei->n_rows, stream, ei->n_codes, p, out, info, esc, &s_cnt);
    else
        section_pass<T, B, 0>(in, nx, ny, nz, rows, ei->n_rows, stream, ei->n_codes, p, out, info, esc, &s_cnt);
    __syncthreads();
    if (threadIdx.x == 0) esc.count[blockIdx.x] = s_cnt;
}

// The listed escapes, a thread each: the row search, the voxel, its level.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_section_escapes(const T* __restrict__ in, int64_t nx, int64_t ny,
                                                            int64_t nz, const roix_quant_info* __restrict__ qi,
                                                            const roix_extract_info* __restrict__ ei,
                                                            const roix_row* __restrict__ rows,
                                                            uint8_t* __restrict__ out, roix_section_info* info,
                                                            SecEsc esc) {
    if (info->status != ROIX_OK) return;
    const SecParams p = sec_params(qi);
    const uint64_t nr = ei->n_rows;
    for (uint32_t w = blockIdx.x; w < esc.ngroups; w += gridDim.x) {  // workgroup w's part of the list
        const unsigned long long cnt = esc.count[w], m = cnt < esc.per ? cnt : esc.per;
        for (unsigned long long i = threadIdx.x; i < m; i += blockDim.x) {
            const uint64_t c = esc.list[(unsigned long long)w * esc.per + i];
            out[c] = (uint8_t)sec_escape(in, nx, ny, nz, rows, nr, c, p, info);
        }
    }
}

template <typename T, int B>
static hipError_t launch_section_w(const LaunchCtx& lc, const T* in, const Geom& g, const roix_fused_out* o,
                                   uint8_t* out, roix_section_info* info, const SecEsc& esc) {
    // one workgroup per resident slot: every workgroup takes the same share
    // of the grid-stride loop, so a grid of whole residency rounds keeps the
    // last round from running on a fraction of the chip
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_section<T, B>, kBlock, 0);
    if (e != hipSuccess) return e;
    int wgs = lc.cus > 0 && per_cu > 0 ? lc.cus * per_cu : lc.grid_stream;
    wgs = wgs < (int)esc.ngroups ? wgs : (int)esc.ngroups;  // a part of the escape list each
    hipLaunchKernelGGL((k_section<T, B>), dim3(wgs), dim3(kBlock), 0, lc.stream, in, g.nx, g.ny, g.nz, o->d_qinfo,
                       o->d_einfo, o->d_rows, (const uint8_t*)o->d_stream, out, info, esc);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_section_t(const LaunchCtx& lc, const T* in, const Geom& g, const roix_fused_out* o,
                                   uint8_t* out, roix_section_info* info, const SecEsc& esc) {
    hipError_t e;
    if ((e = launch_section_w<T, 2>(lc, in, g, o, out, info, esc)) != hipSuccess) return e;
    if ((e = launch_section_w<T, 1>(lc, in, g, o, out, info, esc)) != hipSuccess) return e;
    if ((e = launch_section_w<T, 4>(lc, in, g, o, out, info, esc)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_section_escapes<T>, dim3(esc.ngroups), dim3(kBlock), 0, lc.stream, in, g.nx, g.ny, g.nz,
                       o->d_qinfo, o->d_einfo, o->d_rows, out, info, esc);
    return hipGetLastError();
}

constexpr uint32_t kSecGroups = 4096;  // at most this many workgroups of the streaming pass (one count each)

size_t section_scratch_bytes() { return (size_t)kSecGroups * 8; }

hipError_t launch_section(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g,
                          const roix_fused_out* o, uint8_t* out, int64_t out_cap, roix_section_info* info,
                          void* scratch, size_t scratch_bytes) {
    SecEsc esc;
    esc.ngroups = kSecGroups;
    esc.count = (unsigned long long*)scratch;
    esc.list = (unsigned long long*)((uint8_t*)scratch + section_scratch_bytes());
    esc.per = scratch_bytes > section_scratch_bytes() ? (scratch_bytes - section_scratch_bytes()) / 8 / kSecGroups : 0;
    timer_begin(lc.timer, ST_SECTION, lc.stream);
    hipLaunchKernelGGL(k_section_check, dim3(1), dim3(256), 0, lc.stream, o->d_qinfo, o->d_einfo, o->rows_cap,
                       o->stream_cap_bytes, out_cap, info, esc);
    const hipError_t e = dt == ROIX_F32 ? launch_section_t(lc, (const float*)in, g, o, out, info, esc)
                                        : launch_section_t(lc, (const uint16_t*)in, g, o, out, info, esc);
    timer_end(lc.timer, ST_SECTION, lc.stream);
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace roix
