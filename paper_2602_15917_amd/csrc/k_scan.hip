// k_scan.hip - exclusive prefix sums with a fixed workgroup count.
//
// Reduce-then-scan in three launches: kScanBlocks workgroups each reduce one
// contiguous chunk, one workgroup scans the chunk sums, then every workgroup
// rescans its chunk with its offset.  The element count may live in device
// memory (the number of runs is only known on the device), so the grid never
// depends on data and the whole sequence needs no host synchronisation.
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

template <typename T>
__device__ __forceinline__ void k_scan_reduce_body(const VPart vp, const T* __restrict__ in, int64_t n_host,
                                                        const uint32_t* n_dev, uint64_t* tmp) {
    const int64_t n = scan_n(n_host, n_dev);
    const int64_t chunk = (n + vp.n - 1) / vp.n;
    const int64_t lo = (int64_t)vp.b * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    uint64_t s = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += (uint64_t)in[i];
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

// one workgroup of kScanBlocks threads over the G <= kScanBlocks chunk sums
template <typename TT>
__device__ __forceinline__ void k_scan_top_body(const VPart vp, uint64_t* tmp, TT* total_out, TT* out_end, DevState* cS,
                                                          uint64_t cap, int cerr, int G) {
    __shared__ uint64_t s[kScanBlocks];
    const int t = threadIdx.x;
    const uint64_t mine = t < G ? tmp[t] : 0ull;
    s[t] = mine;
    __syncthreads();
    for (int o = 1; o < kScanBlocks; o <<= 1) {
        uint64_t a = t >= o ? s[t - o] : 0ull;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint64_t incl = s[t];
    if (t < G) tmp[t] = incl - mine;  // exclusive
    if (t == kScanBlocks - 1) {
        tmp[kScanBlocks] = incl;
        if (total_out) *total_out = (TT)incl;
        if (out_end) *out_end = (TT)incl;
        if (cS && incl > cap) fail(cS, cerr);
    }
}
template <typename TT>
__global__ __launch_bounds__(kScanBlocks) void k_scan_top(uint64_t* tmp, TT* total_out, TT* out_end, DevState* cS,
                                                          uint64_t cap, int cerr, int G) {
    k_scan_top_body<TT>(hw_part(), tmp, total_out, out_end, cS, cap, cerr, G);
}

// As k_scan_top, continuing from a device base: every offset is shifted by
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

template <typename T>
__device__ __forceinline__ void k_scan_down_body(const VPart vp, const T* in, T* out, int64_t n_host, const uint32_t* n_dev,
                                                      const uint64_t* tmp) {
    const int64_t n = scan_n(n_host, n_dev);
    const int64_t chunk = (n + vp.n - 1) / vp.n;
    const int64_t lo = (int64_t)vp.b * chunk;
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
__global__ __launch_bounds__(kBlock) void k_scan_down(const T* in, T* out, int64_t n_host, const uint32_t* n_dev,
                                                      const uint64_t* tmp) {
    k_scan_down_body<T>(hw_part(), in, out, n_host, n_dev, tmp);
}

// the chunk count of a scan: kScanBlocks, or fewer for a batch's small volumes
static int scan_grid(const LaunchCtx& lc) {
    return lc.scan_grid >= 1 && lc.scan_grid <= kScanBlocks ? lc.scan_grid : kScanBlocks;
}

hipError_t launch_scan_u32(const LaunchCtx& lc, const uint32_t* in, uint32_t* out, int64_t n_host,
                           const uint32_t* n_dev, uint32_t* total_out, uint32_t* out_end, uint64_t* tmp,
                           DevState* cap_S, uint64_t cap, int cap_err) {
    timer_begin(lc.timer, ST_SCAN, lc.stream);
    const int G = scan_grid(lc);
    launch_k<kBlock, k_scan_reduce_body<uint32_t>>(lc, k_scan_reduce<uint32_t>, dim3(G), dim3(kBlock), 0, in,
                                                   n_host, n_dev, tmp);
    launch_k<kScanBlocks, k_scan_top_body<uint32_t>>(lc, k_scan_top<uint32_t>, dim3(1), dim3(kScanBlocks), 0, tmp,
                                                     total_out, out_end, cap_S, cap, cap_err, G);
    launch_k<kBlock, k_scan_down_body<uint32_t>>(lc, k_scan_down<uint32_t>, dim3(G), dim3(kBlock), 0, in, out,
                                                 n_host, n_dev, (const uint64_t*)tmp);
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
    hipLaunchKernelGGL(k_scan_down<uint32_t>, dim3(kScanBlocks), dim3(kBlock), 0, lc.stream, in, out, n_host,
                       (const uint32_t*)nullptr, (const uint64_t*)tmp);
    timer_end(lc.timer, ST_SCAN, lc.stream);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const LaunchCtx& lc, const uint64_t* in, uint64_t* out, int64_t n_host,
                           unsigned long long* total_out, uint64_t* tmp) {
    timer_begin(lc.timer, ST_SCAN, lc.stream);
    const int G = scan_grid(lc);
    launch_k<kBlock, k_scan_reduce_body<uint64_t>>(lc, k_scan_reduce<uint64_t>, dim3(G), dim3(kBlock), 0, in,
                                                   n_host, (const uint32_t*)nullptr, tmp);
    launch_k<kScanBlocks, k_scan_top_body<unsigned long long>>(lc, k_scan_top<unsigned long long>, dim3(1),
                                                               dim3(kScanBlocks), 0, tmp, total_out,
                                                               (unsigned long long*)nullptr, (DevState*)nullptr, 0ull,
                                                               0, G);
    launch_k<kBlock, k_scan_down_body<uint64_t>>(lc, k_scan_down<uint64_t>, dim3(G), dim3(kBlock), 0, in, out,
                                                 n_host, (const uint32_t*)nullptr, (const uint64_t*)tmp);
    timer_end(lc.timer, ST_SCAN, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
