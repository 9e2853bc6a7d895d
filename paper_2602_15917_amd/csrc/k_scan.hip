// k_scan.hip - exclusive prefix sums with a fixed workgroup count.
//
// Reduce-then-scan in two launches: G <= kScanBlocks workgroups each reduce
// one contiguous chunk, then every workgroup sums the chunk sums before its
// own (at most kScanBlocks - 1 of them, read from L2) and rescans its chunk
// from that offset; the last workgroup also writes the total.  The element
// count may live in device memory (the number of runs is only known on the
// device), so the grid never depends on data and the whole sequence needs no
// host synchronisation.  Chunks are whole multiples of 4 elements and a
// thread takes 4 consecutive elements a step, so a workgroup covers 1024
// elements with one round of loads.
#include "common.h"

namespace roix {

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_w, T& total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    T x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_w[w] = x;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) {
        T t = s_w[k];
        off += k < w ? t : (T)0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// a device count never exceeds the host bound (the arrays' capacity), even
// when an earlier stage has failed and left the count meaningless
__device__ __forceinline__ int64_t scan_n(int64_t n_host, const uint32_t* n_dev) {
    if (!n_dev) return n_host;
    const int64_t n = (int64_t)(*n_dev);
    return n < n_host ? n : n_host;
}

constexpr int kScanPer = 4;  // consecutive elements per thread and step

// chunk of a scan of n elements over G workgroups: a multiple of kScanPer
__device__ __forceinline__ int64_t scan_chunk(int64_t n, uint32_t G) {
    const int64_t c = (n + G - 1) / G;
    return (c + kScanPer - 1) / kScanPer * kScanPer;
}

template <typename T>
__device__ __forceinline__ void k_scan_reduce_body(const VPart vp, const T* __restrict__ in, int64_t n_host,
                                                        const uint32_t* n_dev, uint64_t* tmp) {
    const int64_t n = scan_n(n_host, n_dev);
    const int64_t chunk = scan_chunk(n, vp.n);
    const int64_t lo = (int64_t)vp.b * chunk < n ? (int64_t)vp.b * chunk : n;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    uint64_t s = 0;
    for (int64_t i0 = lo + kScanPer * threadIdx.x; i0 < hi; i0 += kScanPer * blockDim.x) {
        T v[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) v[k] = i0 + k < hi ? in[i0 + k] : (T)0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) s += (uint64_t)v[k];
    }
    s = wave_sum(s);
    __shared__ uint64_t s_w[kBlock / kWave];
    if (threadIdx.x % kWave == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t += s_w[k];
        tmp[vp.b] = t;
    }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T* __restrict__ in, int64_t n_host,
                                                        const uint32_t* n_dev, uint64_t* tmp) {
    k_scan_reduce_body<T>(hw_part(), in, n_host, n_dev, tmp);
}

// The top level of the streamed-slab scan, continuing from a device base: every offset is shifted by
// *base, then *lo_out = the old base and *base = *out_end = base + total.
__global__ __launch_bounds__(kScanBlocks) void k_scan_top_base(uint64_t* tmp, uint32_t* base, uint32_t* lo_out,
                                                              uint32_t* out_end, DevState* cS, uint64_t cap,
                                                              int cerr) {
    __shared__ uint64_t s[kScanBlocks];
    const int t = threadIdx.x;
    const uint64_t b0 = *base;
    s[t] = tmp[t];
    __syncthreads();
    for (int o = 1; o < kScanBlocks; o <<= 1) {
        uint64_t a = t >= o ? s[t - o] : 0ull;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    const uint64_t incl = s[t];
    tmp[t] = b0 + incl - tmp[t];
    __syncthreads();  // every thread has read *base before it changes
    if (t == kScanBlocks - 1) {
        const uint64_t tot = b0 + incl;
        tmp[kScanBlocks] = tot;
        *lo_out = (uint32_t)b0;
        *base = (uint32_t)tot;
        if (out_end) *out_end = (uint32_t)tot;
        if (cS && tot > cap) fail(cS, cerr);
    }
}

// The sum of tmp[0 .. b) (chunk sums before chunk b, b < kScanBlocks), by
// the whole workgroup of kBlock threads.
__device__ __forceinline__ uint64_t chunk_offset(const uint64_t* tmp, uint32_t b) {
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanBlocks / kBlock; ++k) {
        const uint32_t i = threadIdx.x + (uint32_t)(k * kBlock);
        s += i < b ? tmp[i] : 0ull;
    }
    s = wave_sum(s);
    __shared__ uint64_t s_w[kBlock / kWave];
    if (threadIdx.x % kWave == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) t += s_w[k];
    __syncthreads();
    return t;
}

// Thread t of a step holds elements i0 .. i0 + 3 (i0 = base + 4 t); their
// exclusive offsets start at carry + the scan of the threads' sums.  With
// ci.comps, an element that is a root flag of 1 also writes the entry of
// its component.
template <typename T, typename TT>
__device__ __forceinline__ void k_scan_down_body(const VPart vp, const T* in, T* out, int64_t n_host, const uint32_t* n_dev,
                                                      const uint64_t* tmp, TT* total_out, TT* out_end, DevState* cS,
                                                      uint64_t cap, int cerr, CompInit ci) {
    const int64_t n = scan_n(n_host, n_dev);
    const int64_t chunk = scan_chunk(n, vp.n);
    const int64_t lo = (int64_t)vp.b * chunk < n ? (int64_t)vp.b * chunk : n;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    __shared__ T s_w[kBlock / kWave];
    const uint64_t off = chunk_offset(tmp, vp.b);
    const bool roots = ci.comps && cS && __hip_atomic_load(&cS->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    T carry = (T)off;
    for (int64_t base = lo; base < hi; base += kScanPer * blockDim.x) {
        const int64_t i0 = base + kScanPer * threadIdx.x;
        T v[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) v[k] = i0 + k < hi ? in[i0 + k] : (T)0;
        T s4 = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) s4 += v[k];
        T tot;
        T e = carry + block_excl_scan<T>(s4, s_w, tot);
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = i0 + k;
            if (i < hi) {
                out[i] = e;
                if (roots && v[k] && (uint64_t)e < ci.cap) {
                    roix_component* c = ci.comps + e;
                    c->label = (uint64_t)ci.run_row[i] * (uint64_t)ci.nx + ci.xs[i];
                    c->size = 0;
                    c->x0 = c->y0 = c->z0 = 0xFFFFFFFFu;
                    c->x1 = c->y1 = c->z1 = 0u;
                    c->kept = 0u;
                    c->pad = 0u;
                    ci.kept_flag[e] = 0;
                }
            }
            e += v[k];
        }
        carry += tot;
    }
    if (vp.b == vp.n - 1 && threadIdx.x == 0) {  // the last chunk: the total
        const uint64_t total = off + tmp[vp.b];
        if (total_out) *total_out = (TT)total;
        if (out_end) *out_end = (TT)total;
        if (cS && total > cap) fail(cS, cerr);
    }
}
template <typename T, typename TT>
__global__ __launch_bounds__(kBlock) void k_scan_down(const T* in, T* out, int64_t n_host, const uint32_t* n_dev,
                                                      const uint64_t* tmp, TT* total_out, TT* out_end, DevState* cS,
                                                      uint64_t cap, int cerr, CompInit ci) {
    k_scan_down_body<T, TT>(hw_part(), in, out, n_host, n_dev, tmp, total_out, out_end, cS, cap, cerr, ci);
}

// The same continuing from a device base (streamed slabs): every offset is
// shifted by *base, then *lo_out = the old base and *base = *out_end =
// base + total (one workgroup after the chunk sums).
template <typename T>
__device__ __forceinline__ void k_scan_down_plain_body(const VPart vp, const T* in, T* out, int64_t n_host,
                                                            const uint64_t* tmp) {
    const int64_t n = n_host;
    const int64_t chunk = scan_chunk(n, vp.n);
    const int64_t lo = (int64_t)vp.b * chunk < n ? (int64_t)vp.b * chunk : n;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    __shared__ T s_w[kBlock / kWave];
    T carry = (T)tmp[vp.b];
    for (int64_t base = lo; base < hi; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        T v = i < hi ? in[i] : (T)0;
        T tot;
        T e = block_excl_scan<T>(v, s_w, tot);
        if (i < hi) out[i] = carry + e;
        carry += tot;
    }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_down_plain(const T* in, T* out, int64_t n_host, const uint64_t* tmp) {
    k_scan_down_plain_body<T>(hw_part(), in, out, n_host, tmp);
}

// the chunk count of a scan of at most n_host elements: one workgroup step
// (kScanPer * kBlock elements) a chunk or more, at most kScanBlocks (and at
// most lc.scan_grid), so that a small volume (or each volume of a batch)
// launches only the workgroups it can use
static int scan_grid(const LaunchCtx& lc, int64_t n_host) {
    const int cap = lc.scan_grid >= 1 && lc.scan_grid <= kScanBlocks ? lc.scan_grid : kScanBlocks;
    const int64_t per = (int64_t)kScanPer * kBlock;
    const int64_t need = (n_host + per - 1) / per;
    return need < 1 ? 1 : (need < cap ? (int)need : cap);
}

hipError_t launch_scan_u32(const LaunchCtx& lc, const uint32_t* in, uint32_t* out, int64_t n_host,
                           const uint32_t* n_dev, uint32_t* total_out, uint32_t* out_end, uint64_t* tmp,
                           DevState* cap_S, uint64_t cap, int cap_err, const CompInit* ci) {
    timer_begin(lc.timer, ST_SCAN, lc.stream);
    const int G = scan_grid(lc, n_host);
    const CompInit none{nullptr, nullptr, 0, nullptr, nullptr, 0};
    launch_k<kBlock, k_scan_reduce_body<uint32_t>>(lc, k_scan_reduce<uint32_t>, dim3(G), dim3(kBlock), 0, in,
                                                   n_host, n_dev, tmp);
    launch_k<kBlock, k_scan_down_body<uint32_t, uint32_t>>(lc, k_scan_down<uint32_t, uint32_t>, dim3(G), dim3(kBlock), 0,
                                                           in, out, n_host, n_dev, (const uint64_t*)tmp, total_out,
                                                           out_end, cap_S, cap, cap_err, ci ? *ci : none);
    timer_end(lc.timer, ST_SCAN, lc.stream);
    return hipGetLastError();
}

// (streamed slabs only: always the full chunk count)
hipError_t launch_scan_u32_base(const LaunchCtx& lc, const uint32_t* in, uint32_t* out, int64_t n_host,
                                uint32_t* base, uint32_t* lo_out, uint32_t* out_end, uint64_t* tmp,
                                DevState* cap_S, uint64_t cap, int cap_err) {
    timer_begin(lc.timer, ST_SCAN, lc.stream);
    hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3(kScanBlocks), dim3(kBlock), 0, lc.stream, in, n_host,
                       (const uint32_t*)nullptr, tmp);
    hipLaunchKernelGGL(k_scan_top_base, dim3(1), dim3(kScanBlocks), 0, lc.stream, tmp, base, lo_out, out_end, cap_S,
                       cap, cap_err);
    hipLaunchKernelGGL(k_scan_down_plain<uint32_t>, dim3(kScanBlocks), dim3(kBlock), 0, lc.stream, in, out, n_host,
                       (const uint64_t*)tmp);
    timer_end(lc.timer, ST_SCAN, lc.stream);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const LaunchCtx& lc, const uint64_t* in, uint64_t* out, int64_t n_host,
                           unsigned long long* total_out, uint64_t* tmp) {
    timer_begin(lc.timer, ST_SCAN, lc.stream);
    const int G = scan_grid(lc, n_host);
    launch_k<kBlock, k_scan_reduce_body<uint64_t>>(lc, k_scan_reduce<uint64_t>, dim3(G), dim3(kBlock), 0, in,
                                                   n_host, (const uint32_t*)nullptr, tmp);
    launch_k<kBlock, k_scan_down_body<uint64_t, unsigned long long>>(
        lc, k_scan_down<uint64_t, unsigned long long>, dim3(G), dim3(kBlock), 0, in, out, n_host,
        (const uint32_t*)nullptr, (const uint64_t*)tmp, total_out, (unsigned long long*)nullptr, (DevState*)nullptr,
        0ull, 0, CompInit{nullptr, nullptr, 0, nullptr, nullptr, 0});
    timer_end(lc.timer, ST_SCAN, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
