// k_quant.hip - range, quantiser resolution, codes, histogram + bin proxy, Otsu.
//
// Streaming kernels read the volume with 16-byte loads, one contiguous
// 256 x 16 B x kUnroll block slice per workgroup iteration, grid-stride over
// the volume.  Misaligned heads/tails (volume pointer not 16-byte aligned or
// N not a multiple of the vector width) are handled element-wise.
#include "common.h"

namespace roix {

constexpr int kUnroll = 4;

template <typename T>
struct VecN;
template <>
struct VecN<float> {
    static constexpr int n = 4;
};
template <>
struct VecN<uint16_t> {
    static constexpr int n = 8;
};
template <>
struct VecN<int32_t> {
    static constexpr int n = 4;
};

template <typename T>
__device__ __forceinline__ void unpack16(uint4 raw, T (&v)[VecN<T>::n]);
template <>
__device__ __forceinline__ void unpack16<float>(uint4 raw, float (&v)[4]) {
    v[0] = __uint_as_float(raw.x);
    v[1] = __uint_as_float(raw.y);
    v[2] = __uint_as_float(raw.z);
    v[3] = __uint_as_float(raw.w);
}
template <>
__device__ __forceinline__ void unpack16<int32_t>(uint4 raw, int32_t (&v)[4]) {
    v[0] = (int32_t)raw.x;
    v[1] = (int32_t)raw.y;
    v[2] = (int32_t)raw.z;
    v[3] = (int32_t)raw.w;
}
template <>
__device__ __forceinline__ void unpack16<uint16_t>(uint4 raw, uint16_t (&v)[8]) {
    v[0] = (uint16_t)(raw.x & 0xFFFFu);
    v[1] = (uint16_t)(raw.x >> 16);
    v[2] = (uint16_t)(raw.y & 0xFFFFu);
    v[3] = (uint16_t)(raw.y >> 16);
    v[4] = (uint16_t)(raw.z & 0xFFFFu);
    v[5] = (uint16_t)(raw.z >> 16);
    v[6] = (uint16_t)(raw.w & 0xFFFFu);
    v[7] = (uint16_t)(raw.w >> 16);
}

// Elements [0, head) are before the first 16-byte boundary; vectors cover
// [head, head + nvec * VN); the rest is the tail.
template <typename T>
static void split_vec(const void* p, uint64_t N, uint64_t* head, uint64_t* nvec) {
    constexpr int VN = VecN<T>::n;
    uintptr_t a = (uintptr_t)p;
    uint64_t h = (a % 16) ? (16 - a % 16) / sizeof(T) : 0;
    if (h > N) h = N;
    *head = h;
    *nvec = (N - h) / VN;
}

__device__ __forceinline__ bool block_exit(const DevState* S) {
    __shared__ int s_exit;
    if (threadIdx.x == 0) s_exit = __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    return s_exit != 0;
}

// ------------------------------------------------------------------ init

__device__ bool resolve_bound(double eb, float& eb32, float& w, float& r);

// eb_abs > 0: also the quantiser of that absolute bound (zeros when the bound
// is unusable; the resolve after the range then reports it)
__device__ __forceinline__ void k_init_body(const VPart vp, DevState* S, double eb_abs) {
    {
        if (threadIdx.x == 0) {
            S->status = 0;
            S->trunc = 0;
            S->kmin = 0xFFFFFFFFu;
            S->kmax = 0u;
            S->nonfinite = 0u;
            S->xmin = S->xmax = S->eb32 = S->w = S->r = S->binscale = 0.0f;
            S->qmin = S->qmax = S->width_bits = 0;
            S->esc = 0u;
            S->K = 0;
            S->otsu_bin = -1;
            S->thr_t[0] = S->thr_t[1] = S->thr_t[2] = -1;
            S->n_classes = 0;
            S->q_thr = 0;
            S->proxy_thr = 0;
            S->flags = 0u;
            S->n_mask = 0ull;
            S->n_runs = 0u;
            S->n_comps = 0u;
            S->max_size = 0ull;
            S->largest_cid = kNone;
            S->bbox[0] = S->bbox[2] = S->bbox[4] = 0xFFFFFFFFu;
            S->bbox[1] = S->bbox[3] = S->bbox[5] = 0u;
            S->n_kept = S->n_kept_voxels = 0ull;
            S->span_total = S->n_outliers = S->q_outliers = 0ull;
            S->n_slow = 0u;
            S->p16 = 0u;
            S->qstatus = 0;
            S->seg_lo = 0u;
            S->saved_status = 0;
            S->serve_r = S->serve_rt = 0.0f;
            S->store_used = S->store_slab = 0ull;
            float eb32, w, r;
            if (eb_abs > 0.0 && resolve_bound(eb_abs, eb32, w, r)) {
                S->eb32 = eb32;
                S->w = w;
                S->r = r;
            }
        }
        S->hist[threadIdx.x] = 0ull;
        if (threadIdx.x == 0) {
            S->done_keep = 0u;
            S->kept_root = kNone;
            S->kept_by_root = 0u;
        }
    }
}
__global__ __launch_bounds__(kBlock) void k_init(DevState* S, double eb_abs) {
    k_init_body(hw_part(), S, eb_abs);
}

hipError_t launch_init(const LaunchCtx& lc, DevState* S, double eb_abs) {
    timer_begin(lc.timer, ST_INIT, lc.stream);
    launch_k<kBlock, k_init_body>(lc, k_init, dim3(1), dim3(kBlock), 0, S, eb_abs);
    timer_end(lc.timer, ST_INIT, lc.stream);
    return hipGetLastError();
}

// ----------------------------------------------------------------- range

template <typename T>
__device__ __forceinline__ uint32_t range_key(T x, uint32_t& nonfinite);
template <>
__device__ __forceinline__ uint32_t range_key<float>(float x, uint32_t& nonfinite) {
    uint32_t b = __float_as_uint(x);
    nonfinite |= ((b & 0x7F800000u) == 0x7F800000u) ? 1u : 0u;
    return f2key(x);
}
template <>
__device__ __forceinline__ uint32_t range_key<uint16_t>(uint16_t x, uint32_t& nonfinite) {
    return (uint32_t)x;
}

template <typename T>
__device__ __forceinline__ void k_range_body(const VPart vp, const T* __restrict__ in, uint64_t N, uint64_t head,
                                                  uint64_t nvec, DevState* S) {
    constexpr int VN = VecN<T>::n;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, nf = 0u;
    const uint64_t tid = (uint64_t)vp.b * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)vp.n * blockDim.x;
    // scalar head and tail
    const uint64_t tail0 = head + nvec * VN;
    for (uint64_t i = tid; i < head + (N - tail0); i += nthreads) {
        uint64_t v = i < head ? i : tail0 + (i - head);
        uint32_t k = range_key<T>(in[v], nf);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
    const uint4* vin = reinterpret_cast<const uint4*>(in + head);
    const uint64_t per_iter = nthreads * kUnroll;
    for (uint64_t base = (uint64_t)vp.b * blockDim.x * kUnroll; base < nvec; base += per_iter) {
        uint4 raw[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            uint64_t vi = base + (uint64_t)k * blockDim.x + threadIdx.x;
            raw[k] = vi < nvec ? ld_stream(vin + vi) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            uint64_t vi = base + (uint64_t)k * blockDim.x + threadIdx.x;
            if (vi >= nvec) continue;
            T v[VN];
            unpack16<T>(raw[k], v);
#pragma unroll
            for (int j = 0; j < VN; ++j) {
                uint32_t key = range_key<T>(v[j], nf);
                lo = key < lo ? key : lo;
                hi = key > hi ? key : hi;
            }
        }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    nf = wave_max(nf);
    __shared__ uint32_t s_lo[kBlock / kWave], s_hi[kBlock / kWave], s_nf[kBlock / kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_nf[w] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) {
            lo = s_lo[k] < lo ? s_lo[k] : lo;
            hi = s_hi[k] > hi ? s_hi[k] : hi;
            nf |= s_nf[k];
        }
        atomicMin(&S->kmin, lo);
        atomicMax(&S->kmax, hi);
        if (nf) atomicOr(&S->nonfinite, 1u);
    }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_range(const T* __restrict__ in, uint64_t N, uint64_t head,
                                                  uint64_t nvec, DevState* S) {
    k_range_body<T>(hw_part(), in, N, head, nvec, S);
}

static int stream_grid(const LaunchCtx& lc, uint64_t nvec) {
    uint64_t need = (nvec + (uint64_t)kBlock * kUnroll - 1) / ((uint64_t)kBlock * kUnroll);
    if (need < 1) need = 1;
    return (int)(need < (uint64_t)lc.grid_read ? need : (uint64_t)lc.grid_read);
}

hipError_t launch_range(const LaunchCtx& lc, const void* in, roix_dtype dt, uint64_t N, DevState* S) {
    uint64_t head, nvec;
    timer_begin(lc.timer, ST_RANGE, lc.stream);
    if (dt == ROIX_F32) {
        split_vec<float>(in, N, &head, &nvec);
        launch_k<kBlock, k_range_body<float>>(lc, k_range<float>, dim3(stream_grid(lc, nvec)), dim3(kBlock), 0,
                           (const float*)in, N, head, nvec, S);
    } else {
        split_vec<uint16_t>(in, N, &head, &nvec);
        launch_k<kBlock, k_range_body<uint16_t>>(lc, k_range<uint16_t>, dim3(stream_grid(lc, nvec)), dim3(kBlock), 0,
                           (const uint16_t*)in, N, head, nvec, S);
    }
    timer_end(lc.timer, ST_RANGE, lc.stream);
    return hipGetLastError();
}

// --------------------------------------------------------------- resolve

__device__ __forceinline__ bool is_normal_f32(float f) {
    uint32_t e = (__float_as_uint(f) >> 23) & 0xFFu;
    return e != 0u && e != 0xFFu;
}

// fixed threshold T (input units): object = q > q(T), q(T) clamped to [qmin-1, qmax]
__device__ void resolve_fixed(DevState* S, double T) {
    float tf = (float)T;
    float rq = __builtin_rintf(tf * S->r);
    double qd = (double)rq;
    int64_t qT;
    if (qd < (double)S->qmin - 1.0)
        qT = (int64_t)S->qmin - 1;
    else if (qd > (double)S->qmax)
        qT = S->qmax;
    else
        qT = (int64_t)qd;
    S->q_thr = (int32_t)(qT + 1);
    S->proxy_thr = 0;  // the proxy holds the mask bit itself
    S->flags |= ROIX_FLAG_FIXED_THRESHOLD;
}

__device__ void set_width(DevState* S) {
    S->K = (int64_t)S->qmax - (int64_t)S->qmin + 1;
    S->width_bits = S->K <= 255 ? 8 : (S->K <= 65535 ? 16 : 32);
    S->esc = S->width_bits == 32 ? 0xFFFFFFFFu : ((1u << S->width_bits) - 1u);
    S->binscale = (float)(256.0 / (double)S->K);
    const uint64_t M = ((1ull << 40) + (uint64_t)S->K - 1ull) / (uint64_t)S->K;
    S->bin_mlo = (uint32_t)M;
    S->bin_mhi = (uint32_t)(M >> 32);
    bin24_params((uint64_t)S->K, S->bin_a, S->bin_m24);
}

__device__ __forceinline__ void qfail(DevState* S, int32_t st) {
    S->qstatus = st;
    fail(S, st);
}

// The fp32 bound eb32 (eb rounded toward zero, so that the fp32 guarantee
// implies the binary64 one), the step w = 2 eb32 and r = 1/w correctly
// rounded (the binary64 quotient rounded to binary32: double rounding is
// harmless for division since 53 >= 2*24 + 2).  False when eb is not a
// positive finite number or any of the three is not a normal float.
__device__ bool resolve_bound(double eb, float& eb32, float& w, float& r) {
    if (!(eb > 0.0) || !(eb <= 1.7976931348623157e308)) return false;
    eb32 = (float)eb;
    if ((double)eb32 > eb) eb32 = __uint_as_float(__float_as_uint(eb32) - 1u);  // next float toward zero
    if (!is_normal_f32(eb32)) return false;
    w = eb32 + eb32;
    r = (float)(1.0 / (double)w);
    return is_normal_f32(w) && is_normal_f32(r);
}

// the quantiser from the range (one thread)
__device__ void resolve_core(DevState* S, int is_f32, int eb_mode, double eb_value, int fixed, double fixed_value) {
    if (S->nonfinite) {
        qfail(S, ROIX_EINVAL);
        return;
    }
    float xmin = is_f32 ? key2f(S->kmin) : (float)S->kmin;
    float xmax = is_f32 ? key2f(S->kmax) : (float)S->kmax;
    S->xmin = xmin;
    S->xmax = xmax;
    double eb = eb_mode == ROIX_EB_ABS ? eb_value : eb_value * ((double)xmax - (double)xmin);
    float eb32, w, r;
    if (!resolve_bound(eb, eb32, w, r)) {
        qfail(S, ROIX_EINVAL);
        return;
    }
    S->eb32 = eb32;
    S->w = w;
    S->r = r;
    float qlo = xmin * r, qhi = xmax * r;
    if (!(__builtin_fabsf(qlo) <= 16777216.0f) || !(__builtin_fabsf(qhi) <= 16777216.0f)) {
        qfail(S, ROIX_ERANGE);
        return;
    }
    S->qmin = (int32_t)__builtin_rintf(qlo);
    S->qmax = (int32_t)__builtin_rintf(qhi);
    set_width(S);
    if (fixed) resolve_fixed(S, fixed_value);
}

__device__ __forceinline__ void k_resolve_body(const VPart vp, DevState* S, int is_f32, int eb_mode, double eb_value, int fixed, double fixed_value) {
    if (threadIdx.x != 0 || vp.b != 0) return;
    resolve_core(S, is_f32, eb_mode, eb_value, fixed, fixed_value);
}
__global__ __launch_bounds__(1024) void k_resolve(DevState* S, int is_f32, int eb_mode, double eb_value, int fixed, double fixed_value) {
    k_resolve_body(hw_part(), S, is_f32, eb_mode, eb_value, fixed, fixed_value);
}

hipError_t launch_resolve_dt(const LaunchCtx& lc, DevState* S, roix_dtype dt, roix_eb eb,
                             const roix_criterion* crit) {
    int fixed = crit && crit->thr == ROIX_THR_FIXED;
    timer_begin(lc.timer, ST_RESOLVE, lc.stream);
    launch_k<1024, k_resolve_body>(lc, k_resolve, dim3(1), dim3(64), 0, S, dt == ROIX_F32 ? 1 : 0, (int)eb.mode,
                       eb.value, fixed, fixed ? crit->fixed_value : 0.0);
    timer_end(lc.timer, ST_RESOLVE, lc.stream);
    return hipGetLastError();
}

// segment from codes: the quantiser comes from a quant info written earlier
__global__ void k_seg_init(DevState* S, const roix_quant_info* qi, int fixed, double fixed_value) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (qi->status != 0) {
        fail(S, qi->status);
        return;
    }
    S->xmin = qi->xmin;
    S->xmax = qi->xmax;
    S->eb32 = qi->eb32;
    S->w = qi->w;
    S->r = qi->r;
    S->qmin = qi->qmin;
    S->qmax = qi->qmax;
    if (qi->qmax < qi->qmin || !is_normal_f32(qi->w) || !is_normal_f32(qi->r)) {
        fail(S, ROIX_EINVAL);
        return;
    }
    set_width(S);
    if (fixed) resolve_fixed(S, fixed_value);
}

hipError_t launch_seg_init(const LaunchCtx& lc, DevState* S, const roix_quant_info* qinfo,
                           const roix_criterion* crit) {
    int fixed = crit->thr == ROIX_THR_FIXED;
    timer_begin(lc.timer, ST_RESOLVE, lc.stream);
    hipLaunchKernelGGL(k_seg_init, dim3(1), dim3(64), 0, lc.stream, S, qinfo, fixed,
                       fixed ? crit->fixed_value : 0.0);
    timer_end(lc.timer, ST_RESOLVE, lc.stream);
    return hipGetLastError();
}

// -------------------------------------------------------- standalone codes

template <typename T>
__global__ __launch_bounds__(kBlock) void k_quantize(const T* __restrict__ in, uint64_t N, DevState* S,
                                                     int32_t* __restrict__ codes, uint32_t* __restrict__ bits) {
    if (block_exit(S)) return;
    const float r = S->r, w = S->w, eb32 = S->eb32;
    const int lane = threadIdx.x % kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
    uint32_t cnt = 0;
    for (uint64_t b = wave * kWave; b < N; b += nwaves * kWave) {
        uint64_t v = b + lane;
        bool o = false;
        if (v < N) {
            float x = (float)in[v];
            int32_t q = qcode(x, r);
            o = outlier(x, q, w, eb32);
            codes[v] = q;
        }
        uint64_t m = __ballot(o);
        if (lane == 0) {
            cnt += (uint32_t)__popcll(m);
            if (bits) {
                bits[b / 32] = (uint32_t)m;
                if (b + 32 < N) bits[b / 32 + 1] = (uint32_t)(m >> 32);
            }
        }
    }
    if (lane == 0 && cnt) atomicAdd(&S->q_outliers, (unsigned long long)cnt);
}

hipError_t launch_quantize(const LaunchCtx& lc, const void* in, roix_dtype dt, uint64_t N, DevState* S,
                           int32_t* codes, uint32_t* outlier_bits) {
    uint64_t need = (N + kBlock - 1) / kBlock;
    int g = (int)(need < (uint64_t)lc.grid_stream * 4 ? need : (uint64_t)lc.grid_stream * 4);
    if (g < 1) g = 1;
    timer_begin(lc.timer, ST_QUANTIZE, lc.stream);
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_quantize<float>, dim3(g), dim3(kBlock), 0, lc.stream, (const float*)in, N, S, codes,
                           outlier_bits);
    else
        hipLaunchKernelGGL(k_quantize<uint16_t>, dim3(g), dim3(kBlock), 0, lc.stream, (const uint16_t*)in, N, S,
                           codes, outlier_bits);
    timer_end(lc.timer, ST_QUANTIZE, lc.stream);
    return hipGetLastError();
}

// ----------------------------------------------- histogram + 1-byte proxy

struct QH {
    float r;
    int32_t qmin, q_thr;
    uint32_t K, mlo, mhi, a24, m24;
    float binscale;
};

// Code -> bin (and object flag for a fixed threshold) of one voxel; the
// histogram count goes to this lane's LDS copy.  Returns the proxy byte.
template <typename T, bool CODES, bool FIXED, int DIV>
__device__ __forceinline__ uint32_t qh_one(T x, const QH& p, uint32_t* lh_copy, bool& bad) {
    int32_t q;
    if constexpr (CODES)
        q = (int32_t)x;
    else
        q = qcode((float)x, p.r);
    uint32_t u = (uint32_t)(q - p.qmin);
    if constexpr (CODES) {
        if (u >= p.K) {
            bad = true;
            u = 0u;
        }
    }
    const uint32_t b = DIV == 2 ? bin24(u, p.a24, p.m24) : (DIV == 1 ? bin_fast(u, p.mlo, p.mhi) : bin_slow(u, p.K, p.binscale));
    atomicAdd(&lh_copy[b], 1u);
    if constexpr (FIXED)
        return q >= p.q_thr ? 1u : 0u;
    else
        return b;
}

constexpr int kQhBatch = 8;  // 16-byte loads in flight per lane

template <typename T, bool CODES, bool FIXED, int DIV>
__device__ __forceinline__ void qh_vec(const uint4& raw, uint8_t* __restrict__ dst, int64_t vi, const QH& p,
                                       uint32_t* mine, bool& bad) {
    constexpr int VN = VecN<T>::n;
    T v[VN];
    unpack16<T>(raw, v);
    if constexpr (VN == 4) {
        uint32_t pk = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) pk |= qh_one<T, CODES, FIXED, DIV>(v[j], p, mine, bad) << (8 * j);
        if (dst) reinterpret_cast<uint32_t*>(dst)[vi] = pk;
    } else {
        uint64_t pk = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) pk |= (uint64_t)qh_one<T, CODES, FIXED, DIV>(v[j], p, mine, bad) << (8 * j);
        if (dst) reinterpret_cast<uint64_t*>(dst)[vi] = pk;
    }
}

// Flat path (rows not 16-byte aligned, the volume is): the N values as one
// array of 16-byte vectors, kQhBatch in flight per lane, a wave step being
// kQhSlots consecutive vectors.  A value's row and column come from the
// step's first row and column (one scalar division per step) and its offset
// in the step: q = floor(t / nx) for t < nx + kQhSlots * VN from a float
// estimate and one correction.  The last N mod VN values go value by value.
template <typename T, bool CODES, bool FIXED, int DIV, bool STORE>
__device__ __forceinline__ void qh_flat(const VPart vp, const T* __restrict__ in, int64_t nx, int64_t nrows, int64_t P,
                                        const QH& p, uint32_t* mine, uint8_t* __restrict__ proxy, bool& bad) {
    constexpr int VN = VecN<T>::n;
    constexpr int64_t kQhSlots = (int64_t)kWave * kQhBatch;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)vp.b * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)vp.n * blockDim.x / kWave;
    const int64_t N = nx * nrows, nvec = N / VN;
    const uint4* v4 = reinterpret_cast<const uint4*>(in);
    const float inv_nx = 1.0f / (float)nx;
    const uint32_t unx = (uint32_t)nx;
    for (int64_t s0 = wave * kQhSlots; s0 < nvec; s0 += nwaves * kQhSlots) {
        uint4 raw[kQhBatch];
#pragma unroll
        for (int k = 0; k < kQhBatch; ++k) {
            const int64_t vi = s0 + k * kWave + lane;
            raw[k] = vi < nvec ? ld_stream(v4 + vi) : make_uint4(0, 0, 0, 0);
        }
        const int64_t f0 = s0 * VN;  // first value of the step (uniform)
        const int64_t row0 = f0 / nx, x0 = f0 - row0 * nx;
#pragma unroll
        for (int k = 0; k < kQhBatch; ++k) {
            const int64_t vi = s0 + k * kWave + lane;
            if (vi >= nvec) continue;
            T v[VN];
            unpack16<T>(raw[k], v);
            // row (from row0) and column of the vector's first value, then
            // stepped along value by value
            const uint32_t t0 = (uint32_t)(x0 + (vi - s0) * VN);
            uint32_t q = (uint32_t)((float)t0 * inv_nx);
            if ((uint64_t)q * unx > t0) --q;
            if ((uint64_t)(q + 1) * unx <= t0) ++q;
            uint32_t xc = t0 - q * unx;
#pragma unroll
            for (int j = 0; j < VN; ++j) {
                const uint32_t pb = qh_one<T, CODES, FIXED, DIV>(v[j], p, mine, bad);
                if constexpr (STORE) proxy[(row0 + q) * P + xc] = (uint8_t)pb;
                if (++xc == unx) {
                    xc = 0;
                    ++q;
                }
            }
        }
    }
    if (wave == 0)
        for (int64_t f = nvec * VN + lane; f < N; f += kWave) {
            const int64_t row = f / nx, x = f - row * nx;
            const uint32_t pb = qh_one<T, CODES, FIXED, DIV>(ld_stream(in + f), p, mine, bad);
            if constexpr (STORE) proxy[row * P + x] = (uint8_t)pb;
        }
}

// Vector path (VEC 1: row starts 16-byte aligned): 16-byte vectors, stored as
// one word of proxy bytes at the same voxel offset of the row's proxy.  A
// wave fills kQhSlots vector slots per step: rows of at most kQhSlots / 2
// vectors (padded to a power of two) are taken several at a time, longer rows
// one at a time, so that every lane has kQhBatch loads in flight.
// VEC 2: the flat path above.  VEC 0 (the volume itself not 16-byte
// aligned): lane l takes voxels l, l + 64, ... of one row at a time.
template <typename T, bool CODES, bool FIXED, int DIV, int VEC, bool STORE>
__device__ __forceinline__ void qh_rows(const VPart vp, const T* __restrict__ in, int64_t nx, int64_t nrows, int64_t P,
                                        const QH& p, uint32_t* mine, uint8_t* __restrict__ proxy, bool& bad) {
    constexpr int VN = VecN<T>::n;
    constexpr int64_t kQhSlots = (int64_t)kWave * kQhBatch;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)vp.b * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)vp.n * blockDim.x / kWave;
    if constexpr (VEC == 2) {
        qh_flat<T, CODES, FIXED, DIV, STORE>(vp, in, nx, nrows, P, p, mine, proxy, bad);
    } else if constexpr (VEC == 1) {
        const int64_t nv = nx / VN;
        int lg = 0;
        while ((1ll << lg) < nv) ++lg;
        if ((1ll << lg) < kQhSlots) {
            const int64_t rpi = kQhSlots >> lg;  // rows per step
            for (int64_t row0 = wave * rpi; row0 < nrows; row0 += nwaves * rpi) {
                uint4 raw[kQhBatch];
#pragma unroll
                for (int k = 0; k < kQhBatch; ++k) {
                    const int64_t e = (int64_t)k * kWave + lane;
                    const int64_t row = row0 + (e >> lg), vi = e & ((1ll << lg) - 1);
                    raw[k] = (vi < nv && row < nrows) ? ld_stream(reinterpret_cast<const uint4*>(in + row * nx) + vi)
                                                      : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int k = 0; k < kQhBatch; ++k) {
                    const int64_t e = (int64_t)k * kWave + lane;
                    const int64_t row = row0 + (e >> lg), vi = e & ((1ll << lg) - 1);
                    if (vi >= nv || row >= nrows) continue;
                    qh_vec<T, CODES, FIXED, DIV>(raw[k], STORE ? proxy + row * P : nullptr, vi, p, mine, bad);
                }
            }
        } else {
            for (int64_t row = wave; row < nrows; row += nwaves) {
                const uint4* vs = reinterpret_cast<const uint4*>(in + row * nx);
                uint8_t* dst = STORE ? proxy + row * P : nullptr;
                for (int64_t v0 = 0; v0 < nv; v0 += kQhSlots) {
                    uint4 raw[kQhBatch];
#pragma unroll
                    for (int k = 0; k < kQhBatch; ++k) {
                        const int64_t vi = v0 + k * kWave + lane;
                        raw[k] = vi < nv ? ld_stream(vs + vi) : make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                    for (int k = 0; k < kQhBatch; ++k) {
                        const int64_t vi = v0 + k * kWave + lane;
                        if (vi < nv) qh_vec<T, CODES, FIXED, DIV>(raw[k], dst, vi, p, mine, bad);
                    }
                }
            }
        }
    } else {
        for (int64_t row = wave; row < nrows; row += nwaves) {
            const T* src = in + row * nx;
            uint8_t* dst = proxy + row * P;
            for (int64_t x0 = 0; x0 < nx; x0 += kQhSlots) {
                T v[kQhBatch];
#pragma unroll
                for (int k = 0; k < kQhBatch; ++k) {
                    const int64_t x = x0 + k * kWave + lane;
                    v[k] = x < nx ? ld_stream(src + x) : (T)0;
                }
#pragma unroll
                for (int k = 0; k < kQhBatch; ++k) {
                    const int64_t x = x0 + k * kWave + lane;
                    if (x >= nx) continue;
                    const uint32_t pb = qh_one<T, CODES, FIXED, DIV>(v[k], p, mine, bad);
                    if constexpr (STORE) dst[x] = (uint8_t)pb;
                }
            }
        }
    }
}

constexpr int kQhBlock = 512;  // 8 waves share one set of LDS histogram copies

// unless_p16: nothing to do when the fused pass has already produced the
// 16-bit proxy and the histogram
template <typename T, bool CODES, bool FIXED, int VEC, bool STORE = true>
__device__ __forceinline__ void k_quant_hist_body(const VPart vp, const T* __restrict__ in, int64_t nx, int64_t nrows,
                                                       int64_t P, DevState* S, uint8_t* __restrict__ proxy,
                                                       int unless_p16) {
    __shared__ uint32_t lh[kHistCopies * kHistStride];
    for (int i = threadIdx.x; i < kHistCopies * kHistStride; i += blockDim.x) lh[i] = 0u;
    if (block_exit(S)) return;  // contains a barrier, so lh is zeroed for every thread
    if (unless_p16 && S->p16) return;  // uniform, no barrier below before the flush
    QH p;
    p.r = S->r;
    p.qmin = S->qmin;
    p.q_thr = S->q_thr;
    p.K = (uint32_t)S->K;
    p.mlo = S->bin_mlo;
    p.mhi = S->bin_mhi;
    p.a24 = S->bin_a;
    p.m24 = S->bin_m24;
    p.binscale = S->binscale;
    uint32_t* mine = lh + (threadIdx.x % kHistCopies) * kHistStride;
    bool bad = false;
    if (p.m24)
        qh_rows<T, CODES, FIXED, 2, VEC, STORE>(vp, in, nx, nrows, P, p, mine, proxy, bad);
    else if (p.K <= 65536u)
        qh_rows<T, CODES, FIXED, 1, VEC, STORE>(vp, in, nx, nrows, P, p, mine, proxy, bad);
    else
        qh_rows<T, CODES, FIXED, 0, VEC, STORE>(vp, in, nx, nrows, P, p, mine, proxy, bad);
    if constexpr (CODES) {
        if (bad) fail(S, ROIX_EINVAL);
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const int b = threadIdx.x;
        uint32_t s = 0;
#pragma unroll 8
        for (int c = 0; c < kHistCopies; ++c) s += lh[c * kHistStride + b];
        if (s) atomicAdd(&S->hist[b], (unsigned long long)s);
    }
}
template <typename T, bool CODES, bool FIXED, int VEC, bool STORE = true>
__global__ __launch_bounds__(kQhBlock) void k_quant_hist(const T* __restrict__ in, int64_t nx, int64_t nrows,
                                                       int64_t P, DevState* S, uint8_t* __restrict__ proxy,
                                                       int unless_p16) {
    k_quant_hist_body<T, CODES, FIXED, VEC, STORE>(hw_part(), in, nx, nrows, P, S, proxy, unless_p16);
}

static dim3 qh_grid(const LaunchCtx& lc, const Geom& g) {
    int64_t blocks = (g.nrows + kQhBlock / kWave - 1) / (kQhBlock / kWave);
    const int64_t cap = (int64_t)(lc.grid_vox > 0 ? lc.grid_vox : lc.grid_stream) / 2;  // 4 of 512 threads per CU
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return dim3((unsigned)blocks);
}

// 1: rows 16-byte aligned; 2: the volume aligned, its rows not; 0: neither
template <typename T>
static int qh_path(const void* in, const Geom& g) {
    if ((uintptr_t)in % 16 != 0) return 0;
    return (g.nx * (int64_t)sizeof(T)) % 16 == 0 ? 1 : 2;
}

template <typename T, bool CODES>
static void qh_dispatch(const LaunchCtx& lc, const void* in, const Geom& g, DevState* S, uint8_t* proxy,
                        bool fixed, int unless_p16) {
    dim3 grid = qh_grid(lc, g), block(kQhBlock);
    const int vec = qh_path<T>(in, g);
    const int64_t P = g.W * 64;
#define QH_LAUNCH(F, V)                                                                                        \
    launch_k<kQhBlock, k_quant_hist_body<T, CODES, F, V>>(lc, k_quant_hist<T, CODES, F, V>, grid, block, 0, (const T*)in, g.nx, g.nrows, P, \
                       S, proxy, unless_p16)
    if (fixed) {
        if (vec == 1) QH_LAUNCH(true, 1); else if (vec == 2) QH_LAUNCH(true, 2); else QH_LAUNCH(true, 0);
    } else {
        if (vec == 1) QH_LAUNCH(false, 1); else if (vec == 2) QH_LAUNCH(false, 2); else QH_LAUNCH(false, 0);
    }
#undef QH_LAUNCH
}

hipError_t launch_quant_hist(const LaunchCtx& lc, const void* in, int src_kind, const Geom& g, DevState* S,
                             uint8_t* proxy, bool fixed, bool unless_p16) {
    timer_begin(lc.timer, ST_HIST, lc.stream);
    const int u = unless_p16 ? 1 : 0;
    if (src_kind == 0)
        qh_dispatch<float, false>(lc, in, g, S, proxy, fixed, u);
    else if (src_kind == 1)
        qh_dispatch<uint16_t, false>(lc, in, g, S, proxy, fixed, u);
    else
        qh_dispatch<int32_t, true>(lc, in, g, S, proxy, fixed, u);
    timer_end(lc.timer, ST_HIST, lc.stream);
    return hipGetLastError();
}

template <typename T>
static void hist_only_launch(const LaunchCtx& lc, const void* in, const Geom& g, DevState* S) {
    const int vec = qh_path<T>(in, g);
    const int64_t P = g.W * 64;
    if (vec == 1)
        launch_k<kQhBlock, k_quant_hist_body<T, false, false, 1, false>>(lc, k_quant_hist<T, false, false, 1, false>, qh_grid(lc, g), dim3(kQhBlock), 0, (const T*)in, g.nx, g.nrows, P, S, (uint8_t*)nullptr, 0);
    else if (vec == 2)
        launch_k<kQhBlock, k_quant_hist_body<T, false, false, 2, false>>(lc, k_quant_hist<T, false, false, 2, false>, qh_grid(lc, g), dim3(kQhBlock), 0, (const T*)in, g.nx, g.nrows, P, S, (uint8_t*)nullptr, 0);
    else
        launch_k<kQhBlock, k_quant_hist_body<T, false, false, 0, false>>(lc, k_quant_hist<T, false, false, 0, false>, qh_grid(lc, g), dim3(kQhBlock), 0, (const T*)in, g.nx, g.nrows, P, S, (uint8_t*)nullptr, 0);
}

hipError_t launch_hist_only(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g, DevState* S) {
    timer_begin(lc.timer, ST_HIST, lc.stream);
    if (dt == ROIX_F32)
        hist_only_launch<float>(lc, in, g, S);
    else
        hist_only_launch<uint16_t>(lc, in, g, S);
    timer_end(lc.timer, ST_HIST, lc.stream);
    return hipGetLastError();
}

// ------------------------------------ fused range, codes and 16-bit proxy

// With an absolute bound the quantiser is known before the range, so one pass
// can take the range keys and every voxel's code q together.  The proxy then
// holds the low 15 bits of q and the outlier flag in bit 15, and each
// workgroup counts its voxels by q mod 2^15 in LDS.  When the range turns out
// to span at most 2^15 codes (K <= 2^15), q mod 2^15 identifies q, so the
// 256-bin histogram follows exactly from these counts and the proxy decodes
// as q - qmin = (p - qmin) mod 2^15; otherwise the 1-byte proxy pass runs as
// usual.  Rows start 16-byte aligned and hold a multiple of 4 voxels.

constexpr int kQrThreads = 1024;
constexpr int64_t kQrZb = 8;  // slices sharing one load of a reference plane row

__device__ __forceinline__ void qr_vec(const uint4& raw, uint16_t* __restrict__ dst, int64_t vi, float r, float w,
                                       float eb32, uint32_t* fine, uint32_t& lo, uint32_t& hi, uint32_t& nf) {
    const float x[4] = {__uint_as_float(raw.x), __uint_as_float(raw.y), __uint_as_float(raw.z),
                        __uint_as_float(raw.w)};
    uint32_t p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = range_key<float>(x[j], nf);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
        const int32_t q = qcode(x[j], r);
        p[j] = ((uint32_t)q & (uint32_t)(kQrFine - 1)) | (outlier(x[j], q, w, eb32) ? 0x8000u : 0u);
    }
    st_stream(reinterpret_cast<uint2*>(dst + 4 * vi), make_uint2(p[0] | (p[1] << 16), p[2] | (p[3] << 16)));
    // a wave step of one code (a flat region) is one LDS add instead of
    // 256 adds to the same word
    const uint32_t f0 = p[0] & 0x7FFFu;
    const bool same = (((p[0] ^ p[1]) | (p[0] ^ p[2]) | (p[0] ^ p[3])) & 0x7FFFu) == 0u;
    const uint32_t fs = __builtin_amdgcn_readfirstlane(f0);
    const uint64_t act = __ballot(true);
    if (__ballot(!(same && f0 == fs)) == 0ull) {
        if ((uint32_t)(__ffsll((unsigned long long)act) - 1) == (uint32_t)(threadIdx.x % kWave))
            atomicAdd(&fine[fs], 4u * (uint32_t)__popcll(act));
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) atomicAdd(&fine[p[j] & 0x7FFFu], 1u);
    }
}

// M = I - B lane by lane: the raw bits of 4 image voxels minus 4 reference voxels
__device__ __forceinline__ uint4 qr_sub(const uint4& a, const uint4& b) {
    return make_uint4(__float_as_uint(__uint_as_float(a.x) - __uint_as_float(b.x)),
                      __float_as_uint(__uint_as_float(a.y) - __uint_as_float(b.y)),
                      __float_as_uint(__uint_as_float(a.z) - __uint_as_float(b.z)),
                      __float_as_uint(__uint_as_float(a.w) - __uint_as_float(b.w)));
}

// BG: the pass quantises M = I - B, B read from bg (row r of the image takes
// row r % ny of a plane reference, or row r of a volume reference)
template <bool BG>
__device__ __forceinline__ void k_quant_range16_body(const VPart vp, const float* __restrict__ in, int64_t nx, int64_t nrows,
                                                            int64_t P, DevState* S, uint16_t* __restrict__ proxy,
                                                            uint32_t* __restrict__ slots,
                                                            unsigned long long* __restrict__ fine_total,
                                                            const float* __restrict__ bg, int64_t bg_ny) {
    __shared__ uint32_t fine[kQrFine];
    for (int i = threadIdx.x; i < kQrFine; i += blockDim.x) fine[i] = 0u;
    // this workgroup's share of the totals the reduce adds into
    for (int i = threadIdx.x; i < kQrFine / kQrBlocks; i += blockDim.x)
        fine_total[vp.b * (kQrFine / kQrBlocks) + i] = 0ull;
    if (block_exit(S)) return;  // contains a barrier
    const float r = S->r, w = S->w, eb32 = S->eb32;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, nf = 0u;
    // with a reference each load has a partner: half the batch keeps the
    // registers within the 1024-thread budget
    constexpr int NB = BG ? kQhBatch / 2 : kQhBatch;
    constexpr int64_t kSlots = (int64_t)kWave * NB;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)vp.b * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)vp.n * blockDim.x / kWave;
    const int64_t nv = nx / 4;
    int lg = 0;
    while ((1ll << lg) < nv) ++lg;
    if (BG && bg_ny && (1ll << lg) >= kSlots) {
        // a plane reference on long rows: a wave takes one plane row y and
        // the image rows y of kQrZb consecutive slices, so that each plane
        // row is loaded once per kQrZb slices; the next slice's loads are in
        // flight while one is quantised
        const int64_t ny = bg_ny, nzb = (nrows / ny + kQrZb - 1) / kQrZb;
        for (int64_t u = wave; u < ny * nzb; u += nwaves) {
            const int64_t y = u % ny, z0 = (u / ny) * kQrZb;
            const int64_t z1 = z0 + kQrZb < nrows / ny ? z0 + kQrZb : nrows / ny;
            const uint4* bs = reinterpret_cast<const uint4*>(bg + y * nx);
            for (int64_t v0 = 0; v0 < nv; v0 += kSlots) {
                uint4 braw[NB], cur[NB], nxt[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const int64_t vi = v0 + k * kWave + lane;
                    braw[k] = vi < nv ? bs[vi] : make_uint4(0, 0, 0, 0);
                    cur[k] = vi < nv ? ld_stream(reinterpret_cast<const uint4*>(in + (z0 * ny + y) * nx) + vi)
                                     : make_uint4(0, 0, 0, 0);
                }
                for (int64_t z = z0; z < z1; ++z) {
                    // the next slice's row (the last one repeats, unused)
                    const int64_t zn = z + 1 < z1 ? z + 1 : z;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int64_t vi = v0 + k * kWave + lane;
                        nxt[k] = vi < nv ? ld_stream(reinterpret_cast<const uint4*>(in + (zn * ny + y) * nx) + vi)
                                         : make_uint4(0, 0, 0, 0);
                    }
                    uint16_t* dst = proxy + (z * ny + y) * P;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int64_t vi = v0 + k * kWave + lane;
                        if (vi < nv) qr_vec(qr_sub(cur[k], braw[k]), dst, vi, r, w, eb32, fine, lo, hi, nf);
                    }
#pragma unroll
                    for (int k = 0; k < NB; ++k) cur[k] = nxt[k];
                }
            }
        }
    } else if ((1ll << lg) < kSlots) {  // several rows per step (row lengths padded to a power of two)
        const int64_t rpi = kSlots >> lg;
        for (int64_t row0 = wave * rpi; row0 < nrows; row0 += nwaves * rpi) {
            uint4 raw[NB], braw[BG ? NB : 1];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int64_t e = (int64_t)k * kWave + lane;
                const int64_t row = row0 + (e >> lg), vi = e & ((1ll << lg) - 1);
                const bool ok = vi < nv && row < nrows;
                raw[k] = ok ? ld_stream(reinterpret_cast<const uint4*>(in + row * nx) + vi) : make_uint4(0, 0, 0, 0);
                if constexpr (BG) {
                    const int64_t brow = bg_ny ? row % bg_ny : row;
                    braw[k] = ok ? *(reinterpret_cast<const uint4*>(bg + brow * nx) + vi) : make_uint4(0, 0, 0, 0);
                }
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int64_t e = (int64_t)k * kWave + lane;
                const int64_t row = row0 + (e >> lg), vi = e & ((1ll << lg) - 1);
                if (vi >= nv || row >= nrows) continue;
                if constexpr (BG)
                    qr_vec(qr_sub(raw[k], braw[k]), proxy + row * P, vi, r, w, eb32, fine, lo, hi, nf);
                else
                    qr_vec(raw[k], proxy + row * P, vi, r, w, eb32, fine, lo, hi, nf);
            }
        }
    } else {
        for (int64_t row = wave; row < nrows; row += nwaves) {
            const uint4* vs = reinterpret_cast<const uint4*>(in + row * nx);
            const uint4* bs = BG ? reinterpret_cast<const uint4*>(bg + (bg_ny ? row % bg_ny : row) * nx) : nullptr;
            uint16_t* dst = proxy + row * P;
            for (int64_t v0 = 0; v0 < nv; v0 += kSlots) {
                uint4 raw[NB], braw[BG ? NB : 1];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const int64_t vi = v0 + k * kWave + lane;
                    raw[k] = vi < nv ? ld_stream(vs + vi) : make_uint4(0, 0, 0, 0);
                    if constexpr (BG) braw[k] = vi < nv ? bs[vi] : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const int64_t vi = v0 + k * kWave + lane;
                    if (vi >= nv) continue;
                    if constexpr (BG)
                        qr_vec(qr_sub(raw[k], braw[k]), dst, vi, r, w, eb32, fine, lo, hi, nf);
                    else
                        qr_vec(raw[k], dst, vi, r, w, eb32, fine, lo, hi, nf);
                }
            }
        }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    nf = wave_max(nf);
    if (lane == 0) {
        atomicMin(&S->kmin, lo);
        atomicMax(&S->kmax, hi);
        if (nf) atomicOr(&S->nonfinite, 1u);
    }
    __syncthreads();
    uint32_t* mine = slots + (int64_t)vp.b * kQrFine;
    for (int i = threadIdx.x; i < kQrFine; i += blockDim.x) mine[i] = fine[i];
}
template <bool BG>
__global__ __launch_bounds__(kQrThreads) void k_quant_range16(const float* __restrict__ in, int64_t nx, int64_t nrows,
                                                            int64_t P, DevState* S, uint16_t* __restrict__ proxy,
                                                            uint32_t* __restrict__ slots,
                                                            unsigned long long* __restrict__ fine_total,
                                                            const float* __restrict__ bg, int64_t bg_ny) {
    k_quant_range16_body<BG>(hw_part(), in, nx, nrows, P, S, proxy, slots, fine_total, bg, bg_ny);
}

// fine[i] += the counts of code class i of kReduceSlots workgroups (grid.y
// picks the group of slots; fine was cleared by the pass)
constexpr int kReduceSlots = 32;
// workgroup (x, y) of the kQrFine / 256 x kQrBlocks / kReduceSlots grid is
// workgroup y * (kQrFine / 256) + x of a flat grid
__device__ __forceinline__ void k_fine_reduce_body(const VPart vp, const uint32_t* __restrict__ slots,
                                                   unsigned long long* __restrict__ fine) {
    const uint32_t bx = vp.b % (uint32_t)(kQrFine / 256), by = vp.b / (uint32_t)(kQrFine / 256);
    const int i = (int)bx * blockDim.x + threadIdx.x;
    const uint32_t* src = slots + (int64_t)by * kReduceSlots * kQrFine + i;
    uint32_t c[kReduceSlots];
#pragma unroll
    for (int b = 0; b < kReduceSlots; ++b) c[b] = src[(int64_t)b * kQrFine];
    unsigned long long s = 0;
#pragma unroll
    for (int b = 0; b < kReduceSlots; ++b) s += c[b];
    if (s) atomicAdd(&fine[i], s);
}
__global__ __launch_bounds__(256) void k_fine_reduce(const uint32_t* __restrict__ slots,
                                                     unsigned long long* __restrict__ fine) {
    k_fine_reduce_body(hw_part(), slots, fine);
}

// The 256-bin histogram from code-class counts (K <= 2^15): class i holds
// the code q = qmin + ((i - qmin) mod 2^15).  Only the K classes of codes
// qmin .. qmax can hold voxels; thread t of the 1024 takes a run of
// consecutive codes u = q - qmin.  sh: 256 zeroed shared counters.
__device__ void hist_from_classes(DevState* S, const unsigned long long* __restrict__ fine,
                                  unsigned long long* sh) {
    const int t = threadIdx.x;
    const uint32_t qm = (uint32_t)S->qmin, K = (uint32_t)S->K, mlo = S->bin_mlo, mhi = S->bin_mhi;
    const uint32_t per = (K + 1023u) / 1024u;
    uint32_t cur = 0;
    unsigned long long acc = 0ull;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t u = (uint32_t)t * per + j;
        if (u >= K) break;
        const unsigned long long c = fine[(qm + u) & (uint32_t)(kQrFine - 1)];
        if (c == 0ull) continue;
        const uint32_t b = bin_fast(u, mlo, mhi);
        if (b != cur && acc) {
            atomicAdd(&sh[cur], acc);
            acc = 0ull;
        }
        cur = b;
        acc += c;
    }
    if (acc) atomicAdd(&sh[cur], acc);
    __syncthreads();
    if (t < 256) S->hist[t] = sh[t];
}

// The quantiser from the range, then (K <= 2^15) the 256-bin histogram from
// the class counts.
__device__ __forceinline__ void k_resolve16_body(const VPart vp, DevState* S, double eb_value, int fixed, double fixed_value,
                                                    const unsigned long long* __restrict__ fine) {
    __shared__ unsigned long long sh[256];
    __shared__ int s_ok;
    const int t = threadIdx.x;
    if (t < 256) sh[t] = 0ull;
    if (t == 0) {
        resolve_core(S, 1, ROIX_EB_ABS, eb_value, fixed, fixed_value);
        const bool ok = S->status == 0 && S->K <= (int64_t)kQrFine;
        S->p16 = ok ? 1u : 0u;
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    if (!s_ok) return;  // uniform
    hist_from_classes(S, fine, sh);
}
__global__ __launch_bounds__(1024) void k_resolve16(DevState* S, double eb_value, int fixed, double fixed_value,
                                                    const unsigned long long* __restrict__ fine) {
    k_resolve16_body(hw_part(), S, eb_value, fixed, fixed_value, fine);
}

hipError_t launch_quant_range16(const LaunchCtx& lc, const float* in, const Geom& g, const Layout& L, const BgRef* bg) {
    timer_begin(lc.timer, ST_QR16, lc.stream);
    if (bg)
        launch_k<kQrThreads, k_quant_range16_body<true>>(lc, k_quant_range16<true>, dim3(kQrBlocks), dim3(kQrThreads), 0, in, g.nx, g.nrows,
                           g.W * 64, L.S, reinterpret_cast<uint16_t*>(L.proxy), L.fine_slots, L.fine_total, bg->bg,
                           bg->plane ? g.ny : (int64_t)0);
    else
        launch_k<kQrThreads, k_quant_range16_body<false>>(lc, k_quant_range16<false>, dim3(kQrBlocks), dim3(kQrThreads), 0, in, g.nx, g.nrows,
                           g.W * 64, L.S, reinterpret_cast<uint16_t*>(L.proxy), L.fine_slots, L.fine_total,
                           (const float*)nullptr, (int64_t)0);
    timer_end(lc.timer, ST_QR16, lc.stream);
    return hipGetLastError();
}

hipError_t launch_resolve16(const LaunchCtx& lc, const Layout& L, roix_eb eb, const roix_criterion* crit) {
    const int fixed = crit && crit->thr == ROIX_THR_FIXED;
    timer_begin(lc.timer, ST_RESOLVE, lc.stream);
    static_assert(kQrBlocks % kReduceSlots == 0 && kQrFine % kQrBlocks == 0, "reduce tiling");
    launch_k<256, k_fine_reduce_body>(lc, k_fine_reduce, dim3((kQrFine / 256) * (kQrBlocks / kReduceSlots)),
                                      dim3(256), 0, (const uint32_t*)L.fine_slots, L.fine_total);
    launch_k<1024, k_resolve16_body>(lc, k_resolve16, dim3(1), dim3(1024), 0, L.S, eb.value, fixed,
                       fixed ? crit->fixed_value : 0.0, (const unsigned long long*)L.fine_total);
    timer_end(lc.timer, ST_RESOLVE, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------- streamed volumes

// At open: the mask of a streamed volume is decidable voxel by voxel, since
// the bound is absolute and the threshold fixed.  r as the quantiser's, and
// rint(T r) as a float: for every finite voxel with |x r| <= 2^24 (anything
// else fails the volume at close), rint(x r) > rint(T r) is q > q(T), the
// fixed-threshold mask whatever the clamp of q(T) to [qmin - 1, qmax].  An
// unusable bound leaves r = 0 (empty masks); the close reports the error.
__global__ void k_serve_open(DevState* S, double eb_value, double fixed_value) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float eb32, w, r;
    if (!resolve_bound(eb_value, eb32, w, r)) return;
    S->serve_r = r;
    S->serve_rt = __builtin_rintf((float)fixed_value * r);
}

hipError_t launch_serve_open(const LaunchCtx& lc, DevState* S, double eb_value, double fixed_value) {
    hipLaunchKernelGGL(k_serve_open, dim3(1), dim3(64), 0, lc.stream, S, eb_value, fixed_value);
    return hipGetLastError();
}

// Rows [r0, r1) of a slab: one wave per row, 64 consecutive voxels per
// ballot, so each ballot is one mask word; run starts and counts from the
// word and the previous word's top bit.  Also the value range (as the range
// kernel's keys) and the mask count.  Runs regardless of the status, so that
// the counts are complete whatever fails later (as in the whole-volume path).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_slab_mask(const T* __restrict__ in, int64_t nx, int64_t r0, int64_t r1,
                                                      int64_t W, DevState* S, uint64_t* __restrict__ maskbits,
                                                      uint32_t* __restrict__ row_nruns) {
    constexpr int U = 8;  // words per step (loads in flight per lane)
    const float r = S->serve_r, rt = S->serve_rt;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, nf = 0u;
    unsigned long long nmask = 0;
    for (int64_t row = r0 + wave; row < r1; row += nwaves) {
        const T* src = in + row * nx;
        uint64_t carry = 0;
        uint32_t nr = 0;
        for (int64_t w0 = 0; w0 < W; w0 += U) {
            T v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int64_t x = (w0 + k) * 64 + lane;
                v[k] = x < nx ? ld_stream(src + x) : (T)0;
            }
            uint64_t mine = 0;
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (w0 + k >= W) break;  // uniform
                const bool valid = (w0 + k) * 64 + lane < nx;
                const float xf = (float)v[k];
                if (valid) {
                    const uint32_t key = range_key<T>(v[k], nf);
                    lo = key < lo ? key : lo;
                    hi = key > hi ? key : hi;
                }
                const uint64_t m = __ballot(valid && __builtin_rintf(xf * r) > rt);
                const uint64_t starts = m & ~((m << 1) | carry);
                carry = m >> 63;
                nr += (uint32_t)__popcll(starts);
                nmask += (unsigned long long)__popcll(m);
                if (lane == k) mine = m;
            }
            if (lane < U && w0 + lane < W) maskbits[row * W + w0 + lane] = mine;
        }
        if (lane == 0) row_nruns[row] = nr;
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    nf = wave_max(nf);
    __shared__ uint32_t s_lo[kBlock / kWave], s_hi[kBlock / kWave], s_nf[kBlock / kWave];
    __shared__ unsigned long long s_nm[kBlock / kWave];
    const int wv = threadIdx.x / kWave;
    if (lane == 0) {
        s_lo[wv] = lo;
        s_hi[wv] = hi;
        s_nf[wv] = nf;
        s_nm[wv] = nmask;  // the same value in every lane: counted once per wave
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long nm = 0;
        for (int k = 0; k < kBlock / kWave; ++k) {
            lo = s_lo[k] < lo ? s_lo[k] : lo;
            hi = s_hi[k] > hi ? s_hi[k] : hi;
            nf |= s_nf[k];
            nm += s_nm[k];
        }
        if (lo <= hi) {
            atomicMin(&S->kmin, lo);
            atomicMax(&S->kmax, hi);
        }
        if (nf) atomicOr(&S->nonfinite, 1u);
        if (nm) atomicAdd(&S->n_mask, nm);
    }
}

hipError_t launch_slab_mask(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g, int64_t r0,
                            int64_t r1, const Layout& L) {
    timer_begin(lc.timer, ST_MASK_RUNS, lc.stream);
    int64_t blocks = (r1 - r0 + kBlock / kWave - 1) / (kBlock / kWave);
    if (blocks > lc.grid_stream) blocks = lc.grid_stream;
    if (blocks < 1) blocks = 1;
    if (dt == ROIX_F32)
        hipLaunchKernelGGL(k_slab_mask<float>, dim3((unsigned)blocks), dim3(kBlock), 0, lc.stream, (const float*)in,
                           g.nx, r0, r1, g.W, L.S, L.maskbits, L.row_nruns);
    else
        hipLaunchKernelGGL(k_slab_mask<uint16_t>, dim3((unsigned)blocks), dim3(kBlock), 0, lc.stream,
                           (const uint16_t*)in, g.nx, r0, r1, g.W, L.S, L.maskbits, L.row_nruns);
    timer_end(lc.timer, ST_MASK_RUNS, lc.stream);
    return hipGetLastError();
}

// The close of a streamed volume runs resolve, histogram and threshold over
// the whole volume after the slabs have been labelled: an error the slabs
// hit (run capacity) is held back over those stages and restored after them,
// so that the first reported error is the one the whole-volume path reports.
__global__ void k_serve_status(DevState* S, int save) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (save) {
        S->saved_status = S->status;
        S->status = 0;
    } else if (S->status == 0) {
        S->status = S->saved_status;
    }
}

hipError_t launch_serve_status(const LaunchCtx& lc, DevState* S, int save) {
    hipLaunchKernelGGL(k_serve_status, dim3(1), dim3(64), 0, lc.stream, S, save);
    return hipGetLastError();
}

// ------------------------------ streamed volumes kept as row extents
//
// A uint16 stream with an absolute bound and a fixed threshold whose codes
// can span at most 2^15 values (rint(65535 r) < 2^15) keeps, per row, only
// the values between the row's first and last mask voxel: every span lies
// there, since a span runs from the row's first to its last kept voxel and
// kept voxels are mask voxels.  The histogram, which needs the range of the
// whole volume, is rebuilt at close from counts of the code classes
// q mod 2^15, one-to-one on [qmin, qmax] when K <= 2^15 (as in the one-pass
// flow).

__global__ void k_store_open(DevState* S, unsigned long long* __restrict__ classes) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kQrFine; i += gridDim.x * blockDim.x) classes[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) S->store_used = S->store_slab = 0ull;
}

hipError_t launch_store_open(const LaunchCtx& lc, DevState* S, unsigned long long* classes) {
    hipLaunchKernelGGL(k_store_open, dim3(kQrFine / 256), dim3(256), 0, lc.stream, S, classes);
    return hipGetLastError();
}

// Code classes of n slab values: per-workgroup LDS counters (128 KB, one
// workgroup per CU), 16-byte loads of 8 values, then one atomic add per
// non-zero class and workgroup.  r is the open-time quantiser step.
constexpr int kClassThreads = 1024;
__global__ __launch_bounds__(kClassThreads) void k_slab_classes(const uint16_t* __restrict__ in, uint64_t n,
                                                                const DevState* S,
                                                                unsigned long long* __restrict__ classes) {
    __shared__ uint32_t cnt[kQrFine];
    for (int i = threadIdx.x; i < kQrFine; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    const float r = S->serve_r;
    const uint64_t nvec = n / 8;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint4* v4 = reinterpret_cast<const uint4*>(in);
    for (uint64_t i = gt; i < nvec; i += stride) {
        const uint4 q = ld_stream(v4 + i);
        const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            atomicAdd(&cnt[(uint32_t)qcode((float)(wd[k] & 0xFFFFu), r) & (uint32_t)(kQrFine - 1)], 1u);
            atomicAdd(&cnt[(uint32_t)qcode((float)(wd[k] >> 16), r) & (uint32_t)(kQrFine - 1)], 1u);
        }
    }
    for (uint64_t i = nvec * 8 + gt; i < n; i += stride)
        atomicAdd(&cnt[(uint32_t)qcode((float)in[i], r) & (uint32_t)(kQrFine - 1)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kQrFine; i += blockDim.x)
        if (cnt[i]) atomicAdd(&classes[i], (unsigned long long)cnt[i]);
}

hipError_t launch_slab_classes(const LaunchCtx& lc, const uint16_t* stage, uint64_t n, DevState* S,
                               unsigned long long* classes) {
    uint64_t blocks = (n / 8 + (uint64_t)kClassThreads * 16 - 1) / ((uint64_t)kClassThreads * 16);
    const uint64_t cap = (uint64_t)(lc.grid_read > 0 ? lc.grid_read / 4 : 256);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_slab_classes, dim3((unsigned)blocks), dim3(kClassThreads), 0, lc.stream, stage, n,
                       (const DevState*)S, classes);
    return hipGetLastError();
}

// Extent of each slab row from its runs (run_off after the slab's scan,
// run_xs/run_xe written): [xs of the first run, xe of the last run), or
// empty.  lens[r - r0] = its length, xlo[r] = its start.  Nothing when the
// volume has failed (its runs may be unwritten).
__global__ __launch_bounds__(kBlock) void k_store_extent(const uint32_t* __restrict__ run_off,
                                                         const uint32_t* __restrict__ run_xs,
                                                         const uint32_t* __restrict__ run_xe, uint64_t run_cap,
                                                         int64_t r0, int64_t r1, uint32_t* __restrict__ xlo,
                                                         uint64_t* __restrict__ lens, const DevState* S) {
    const bool dead = __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t a = run_off[r], b = run_off[r + 1];
        uint32_t lo = 0, hi = 0;
        if (!dead && b > a && b <= run_cap) {
            lo = run_xs[a];
            hi = run_xe[b - 1];
        }
        xlo[r] = lo;
        lens[r - r0] = (uint64_t)(hi - lo);
    }
}

// Copy each slab row's extent into the store after the values already there
// (offs: exclusive scan of the lengths; S->store_slab their total), a wave
// per row; row_org[r] = store index of voxel (r, 0).  A store that would
// overflow fails the volume (ROIX_ENOMEM) and copies nothing.
__global__ __launch_bounds__(kBlock) void k_store_copy(const uint16_t* __restrict__ stage, int64_t nx, int64_t r0,
                                                       int64_t r1, const uint32_t* __restrict__ xlo,
                                                       const uint64_t* __restrict__ offs, uint16_t* __restrict__ store,
                                                       uint64_t cap, uint64_t* __restrict__ row_org, DevState* S) {
    if (__hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const uint64_t base = S->store_used, total = S->store_slab;
    if (base + total > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) fail(S, ROIX_ENOMEM);
        return;
    }
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = r0 + wave; r < r1; r += nwaves) {
        const uint64_t o = offs[r - r0];
        const uint64_t end = r + 1 < r1 ? offs[r + 1 - r0] : total;
        const uint32_t lo = xlo[r];
        const uint64_t len = end - o;
        if (lane == 0) row_org[r] = base + o - lo;
        const uint16_t* src = stage + (uint64_t)(r - r0) * (uint64_t)nx + lo;
        uint16_t* dst = store + base + o;
        for (uint64_t j = lane; j < len; j += kWave) dst[j] = src[j];
    }
}

__global__ void k_store_advance(DevState* S, uint64_t cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (S->status == 0 && S->store_used + S->store_slab <= cap) S->store_used += S->store_slab;
}

hipError_t launch_store_rows(const LaunchCtx& lc, const Geom& g, const Layout& L, const uint16_t* stage, int64_t r0,
                             int64_t r1, uint16_t* store, uint64_t cap, uint64_t* row_org, uint64_t* lens) {
    const int64_t nr = r1 - r0;
    int64_t blocks = (nr + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_store_extent, dim3((unsigned)blocks), dim3(kBlock), 0, lc.stream,
                       (const uint32_t*)L.run_off, (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, L.run_cap,
                       r0, r1, L.row_xs, lens, (const DevState*)L.S);
    hipError_t e = launch_scan_u64(lc, lens, lens, nr, &L.S->store_slab, L.scan_tmp);
    if (e != hipSuccess) return e;
    int64_t wblocks = (nr + kBlock / kWave - 1) / (kBlock / kWave);
    if (wblocks > lc.grid_stream) wblocks = lc.grid_stream;
    if (wblocks < 1) wblocks = 1;
    hipLaunchKernelGGL(k_store_copy, dim3((unsigned)wblocks), dim3(kBlock), 0, lc.stream, stage, g.nx, r0, r1,
                       (const uint32_t*)L.row_xs, (const uint64_t*)lens, store, cap, row_org, L.S);
    hipLaunchKernelGGL(k_store_advance, dim3(1), dim3(64), 0, lc.stream, L.S, cap);
    return hipGetLastError();
}

// At close: the quantiser from the slabs' range (uint16 keys), the fixed
// threshold, and the histogram from the class counts.  K <= 2^15 is certain
// (checked at open for the whole uint16 range); a quantiser error (none is
// possible for uint16 values with such a bound) leaves the histogram empty.
__global__ __launch_bounds__(1024) void k_serve_resolve(DevState* S, double eb_value, double fixed_value,
                                                        const unsigned long long* __restrict__ classes) {
    __shared__ unsigned long long sh[256];
    __shared__ int s_ok;
    const int t = threadIdx.x;
    if (t < 256) sh[t] = 0ull;
    if (t == 0) {
        resolve_core(S, 0, ROIX_EB_ABS, eb_value, 1, fixed_value);
        const bool ok = S->status == 0;
        if (ok && S->K > (int64_t)kQrFine) fail(S, ROIX_EDEVICE);
        s_ok = ok && S->K <= (int64_t)kQrFine;
    }
    __syncthreads();
    if (!s_ok) return;  // uniform
    hist_from_classes(S, classes, sh);
}

hipError_t launch_serve_resolve(const LaunchCtx& lc, DevState* S, double eb_value, double fixed_value,
                                const unsigned long long* classes) {
    timer_begin(lc.timer, ST_RESOLVE, lc.stream);
    hipLaunchKernelGGL(k_serve_resolve, dim3(1), dim3(1024), 0, lc.stream, S, eb_value, fixed_value, classes);
    timer_end(lc.timer, ST_RESOLVE, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Otsu

// Otsu (1979) on the 256 bins: maximise W0 W1 (m0 - m1)^2 over the split t
// (class 0 = bins 0..t), first maximum on ties, splits with an empty class
// skipped.  Every thread evaluates one split with the same binary64
// expression and operation order.
__device__ __forceinline__ void k_otsu_body(const VPart vp, DevState* S, int fixed) {
    __shared__ unsigned long long sh_w[256], sh_s[256];
    __shared__ double sh_v[256];
    __shared__ int sh_t[256];
    const int t = threadIdx.x;
    if (block_exit(S)) return;
    unsigned long long h = S->hist[t];
    sh_w[t] = h;
    sh_s[t] = (unsigned long long)t * h;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        unsigned long long aw = t >= o ? sh_w[t - o] : 0ull, as = t >= o ? sh_s[t - o] : 0ull;
        __syncthreads();
        sh_w[t] += aw;
        sh_s[t] += as;
        __syncthreads();
    }
    if (fixed) {
        if (t == 0) S->otsu_bin = -1;
        return;
    }
    const unsigned long long NT = sh_w[255], ST = sh_s[255];
    const unsigned long long W0 = sh_w[t], S0 = sh_s[t], W1 = NT - W0;
    double s = -1.0;
    if (t < 255 && W0 != 0ull && W1 != 0ull) {
        double m0 = (double)S0 / (double)W0;
        double m1 = (double)(ST - S0) / (double)W1;
        double d = m0 - m1;
        s = (((double)W0 * (double)W1) * d) * d;
    }
    sh_v[t] = s;
    sh_t[t] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            double a = sh_v[t], b = sh_v[t + o];
            int ta = sh_t[t], tb = sh_t[t + o];
            if (b > a || (b == a && tb < ta)) {
                sh_v[t] = b;
                sh_t[t] = tb;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        int ts = 255;
        if (sh_v[0] < 0.0)
            S->flags |= ROIX_FLAG_DEGENERATE_HISTOGRAM;
        else
            ts = sh_t[0];
        S->otsu_bin = ts;
        S->proxy_thr = ts;
        S->thr_t[0] = ts;
        S->n_classes = 2;
        long long c = ((long long)(ts + 1) * S->K + 255) / 256;
        S->q_thr = (int32_t)((long long)S->qmin + c);
    }
}
__global__ __launch_bounds__(256) void k_otsu(DevState* S, int fixed) {
    k_otsu_body(hw_part(), S, fixed);
}

hipError_t launch_otsu(const LaunchCtx& lc, DevState* S, bool fixed) {
    timer_begin(lc.timer, ST_OTSU, lc.stream);
    launch_k<256, k_otsu_body>(lc, k_otsu, dim3(1), dim3(256), 0, S, fixed ? 1 : 0);
    timer_end(lc.timer, ST_OTSU, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------ per-slice Otsu

// One workgroup per z-slice (grid-stride over slices): the histogram of the
// slice's 1-byte proxy (bins over the volume's code range) and two-class
// Otsu on it, with the same binary64 expression and first-maximum rule as
// k_otsu.  The slice's threshold bin goes to thr[z]; the mask kernel then
// tests "bin > thr[z]" row by row.  16 copies of the LDS counters keep lanes
// that hold the same bin from colliding.
constexpr int kSliceCopies = 16;

__device__ __forceinline__ void k_slice_otsu_body(const VPart vp, const uint8_t* __restrict__ proxy, int64_t nx, int64_t ny,
                                                    int64_t nz, int64_t P, DevState* S, int32_t* __restrict__ thr,
                                                    int32_t* __restrict__ slice_thr) {
    __shared__ uint32_t h[256 * kSliceCopies];
    __shared__ unsigned long long sh_w[256], sh_s[256];
    __shared__ double sh_v[256];
    __shared__ int sh_t[256];
    if (block_exit(S)) return;  // contains a barrier
    const int t = threadIdx.x;
    const uint32_t copy = (uint32_t)t % kSliceCopies;
    // whole 16-byte vectors per row, then single bytes; a slice holds fewer
    // than 2^32 vectors (ny * nx < 2^33 voxels)
    const uint32_t vpr = (uint32_t)(nx / 16), nvec = (uint32_t)((nx / 16) * ny);
    const int64_t tail = nx % 16;
    const int ln = t % kWave;
    const int64_t wv = t / kWave, nw = 256 / kWave;
    if (vp.b == 0 && t == 0) {
        S->proxy_thr = 127;
        S->q_thr = 0;
        S->otsu_bin = -1;
        S->n_classes = 2;
        atomicOr(&S->flags, ROIX_FLAG_PER_SLICE);
    }
    for (int64_t z = vp.b; z < nz; z += vp.n) {
        const uint8_t* base = proxy + z * ny * P;
        for (int i = t; i < 256 * kSliceCopies; i += 256) h[i] = 0u;
        __syncthreads();
        // the slice's 16-byte vectors, flat (row = i / vpr), 8 loads in flight per lane
        for (uint32_t i0 = (uint32_t)t; i0 < nvec; i0 += 8u * 256u) {
            uint4 q[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t i = i0 + 256u * k;
                const uint32_t r = i < nvec ? i / vpr : 0u, v = i < nvec ? i - r * vpr : 0u;
                q[k] = *reinterpret_cast<const uint4*>(base + (int64_t)r * P + 16 * (int64_t)v);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (i0 + 256u * k >= nvec) continue;
                const uint32_t w[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    atomicAdd(&h[((w[b >> 2] >> (8 * (b & 3))) & 0xFFu) * kSliceCopies + copy], 1u);
            }
        }
        for (int64_t r = wv; r < ny && ln < tail; r += nw)
            atomicAdd(&h[(uint32_t)base[r * P + 16 * vpr + ln] * kSliceCopies + copy], 1u);
        __syncthreads();
        unsigned long long hv = 0ull;
#pragma unroll
        for (int c = 0; c < kSliceCopies; ++c) hv += h[t * kSliceCopies + c];
        sh_w[t] = hv;
        sh_s[t] = (unsigned long long)t * hv;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const unsigned long long aw = t >= o ? sh_w[t - o] : 0ull, as = t >= o ? sh_s[t - o] : 0ull;
            __syncthreads();
            sh_w[t] += aw;
            sh_s[t] += as;
            __syncthreads();
        }
        const unsigned long long NT = sh_w[255], ST = sh_s[255];
        const unsigned long long W0 = sh_w[t], S0 = sh_s[t], W1 = NT - W0;
        double sv = -1.0;
        if (t < 255 && W0 != 0ull && W1 != 0ull) {
            double m0 = (double)S0 / (double)W0;
            double m1 = (double)(ST - S0) / (double)W1;
            double d = m0 - m1;
            sv = (((double)W0 * (double)W1) * d) * d;
        }
        sh_v[t] = sv;
        sh_t[t] = t;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) {
                const double a = sh_v[t], b = sh_v[t + o];
                const int ta = sh_t[t], tb = sh_t[t + o];
                if (b > a || (b == a && tb < ta)) {
                    sh_v[t] = b;
                    sh_t[t] = tb;
                }
            }
            __syncthreads();
        }
        const bool degenerate = sh_v[0] < 0.0;
        const int32_t ts = degenerate ? 255 : sh_t[0];
        if (t == 0) {
            if (degenerate) atomicOr(&S->flags, ROIX_FLAG_DEGENERATE_HISTOGRAM);
            thr[z] = ts;
            if (slice_thr) slice_thr[z] = ts;
        }
        __syncthreads();  // sh_* are reused by the next slice
    }
}
__global__ __launch_bounds__(256) void k_slice_otsu(const uint8_t* __restrict__ proxy, int64_t nx, int64_t ny,
                                                    int64_t nz, int64_t P, DevState* S, int32_t* __restrict__ thr,
                                                    int32_t* __restrict__ slice_thr) {
    k_slice_otsu_body(hw_part(), proxy, nx, ny, nz, P, S, thr, slice_thr);
}

hipError_t launch_slice_otsu(const LaunchCtx& lc, const Geom& g, const uint8_t* proxy, DevState* S, int32_t* thr,
                             int32_t* slice_thr_out) {
    timer_begin(lc.timer, ST_OTSU, lc.stream);
    const int64_t grid = g.nz < 8192 ? g.nz : 8192;
    launch_k<256, k_slice_otsu_body>(lc, k_slice_otsu, dim3((unsigned)grid), dim3(256), 0, proxy, g.nx, g.ny, g.nz, g.W * 64,
                       S, thr, slice_thr_out);
    timer_end(lc.timer, ST_OTSU, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------ multi-level Otsu

// Multi-level Otsu (Liao, Chen & Chung 2001) with K = 3 or 4 classes over
// the 256 bins: the thresholds t1 < .. < t_{K-1} in 0..254 (class k = bins
// t_k + 1 .. t_{k+1}, t_0 = -1, t_K = 255) maximising the between-class
// variance, i.e. sum_k S_k^2 / W_k for the fixed histogram (W_k voxels and
// S_k the bin sum of class k), in binary64 in class order.  Tuples with an
// empty class are skipped; the first maximum in lexicographic order wins:
// every workgroup keeps its best (score, rank), rank = the tuple's
// lexicographic position, and one workgroup picks the highest score with the
// smallest rank.  Pairs (t1, t2) are spread over the grid as p = t1 * 255 +
// t2; for K = 4 the workgroup's chunk c takes t3 over
// max(t2 + 1, 32 c) .. min(254, 32 c + 31), so no thread runs more than 32
// tuples.

__device__ __forceinline__ double mo_term(unsigned long long W, unsigned long long S) {
    const double s = (double)S;
    return (s * s) / (double)W;
}

// (value, rank) pairs: the higher value wins, then the smaller rank
__device__ __forceinline__ void mo_take(double& v, unsigned long long& r, double bv, unsigned long long br) {
    if (bv > v || (bv == v && br < r)) {
        v = bv;
        r = br;
    }
}

__device__ __forceinline__ void mo_reduce(double* sv, unsigned long long* sr, int t) {
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            double v = sv[t];
            unsigned long long r = sr[t];
            mo_take(v, r, sv[t + o], sr[t + o]);
            sv[t] = v;
            sr[t] = r;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void k_multi_search_body(const VPart vp, DevState* S, int classes) {
    __shared__ unsigned long long P[257], Q[257];
    __shared__ double sv[256];
    __shared__ unsigned long long sr[256];
    const int t = threadIdx.x;
    // prefix counts and bin sums: P[i], Q[i] over bins 0 .. i-1 (inclusive
    // scan of the bins in LDS; integer sums, so exact in any order)
    const unsigned long long h = S->hist[t];
    P[t + 1] = h;
    Q[t + 1] = (unsigned long long)t * h;
    if (t == 0) P[0] = Q[0] = 0ull;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned long long a = t >= o ? P[t + 1 - o] : 0ull, b = t >= o ? Q[t + 1 - o] : 0ull;
        __syncthreads();
        P[t + 1] += a;
        Q[t + 1] += b;
        __syncthreads();
    }
    double best = -1.0;
    unsigned long long rank = ~0ull;
    const int p = (vp.b % kMoPairBlocks) * blockDim.x + t;
    const int t1 = p / 255, t2 = p % 255;
    if (classes == 3) {
        if (t1 < t2 && t2 < 255) {
            const unsigned long long W0 = P[t1 + 1], W1 = P[t2 + 1] - P[t1 + 1], W2 = P[256] - P[t2 + 1];
            if (W0 && W1 && W2) {
                const unsigned long long S0 = Q[t1 + 1], S1 = Q[t2 + 1] - Q[t1 + 1], S2 = Q[256] - Q[t2 + 1];
                best = (mo_term(W0, S0) + mo_term(W1, S1)) + mo_term(W2, S2);
                rank = (unsigned long long)p;
            }
        }
    } else if (t1 < t2 && t2 < 254) {
        const int c = vp.b / kMoPairBlocks;
        const int lo = max(t2 + 1, c * kMoChunk), hi = min(255, (c + 1) * kMoChunk);
        const unsigned long long W0 = P[t1 + 1], W1 = P[t2 + 1] - P[t1 + 1];
        const unsigned long long S0 = Q[t1 + 1], S1 = Q[t2 + 1] - Q[t1 + 1];
        if (W0 && W1 && lo < hi) {
            const double a = mo_term(W0, S0) + mo_term(W1, S1);
            for (int t3 = lo; t3 < hi; ++t3) {
                const unsigned long long W2 = P[t3 + 1] - P[t2 + 1], W3 = P[256] - P[t3 + 1];
                if (!W2 || !W3) continue;
                const unsigned long long S2 = Q[t3 + 1] - Q[t2 + 1], S3 = Q[256] - Q[t3 + 1];
                const double v = (a + mo_term(W2, S2)) + mo_term(W3, S3);
                if (v > best) {  // t3 ascending: the first maximum of this pair and chunk
                    best = v;
                    rank = (unsigned long long)p * 255ull + (unsigned long long)t3;
                }
            }
        }
    }
    sv[t] = best;
    sr[t] = rank;
    __syncthreads();
    mo_reduce(sv, sr, t);
    if (t == 0) {
        S->mo_val[vp.b] = sv[0];
        S->mo_rank[vp.b] = sr[0];
    }
}
__global__ __launch_bounds__(256) void k_multi_search(DevState* S, int classes) {
    k_multi_search_body(hw_part(), S, classes);
}

__device__ __forceinline__ void k_multi_pick_body(const VPart vp, DevState* S, int classes, int parts) {
    __shared__ double sv[256];
    __shared__ unsigned long long sr[256];
    const int t = threadIdx.x;
    double v = -1.0;
    unsigned long long r = ~0ull;
    for (int i = t; i < parts; i += 256) mo_take(v, r, S->mo_val[i], S->mo_rank[i]);
    sv[t] = v;
    sr[t] = r;
    __syncthreads();
    mo_reduce(sv, sr, t);
    if (t == 0) {
        if (__hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
        int32_t th[3] = {255, 255, classes == 4 ? 255 : -1};
        if (sv[0] < 0.0) {
            S->flags |= ROIX_FLAG_DEGENERATE_HISTOGRAM;
        } else if (classes == 3) {
            th[0] = (int32_t)(sr[0] / 255ull);
            th[1] = (int32_t)(sr[0] % 255ull);
        } else {
            const unsigned long long pr = sr[0] / 255ull;
            th[0] = (int32_t)(pr / 255ull);
            th[1] = (int32_t)(pr % 255ull);
            th[2] = (int32_t)(sr[0] % 255ull);
        }
        S->thr_t[0] = th[0];
        S->thr_t[1] = th[1];
        S->thr_t[2] = th[2];
        S->n_classes = classes;
        // object: every class above the lowest threshold
        const int ts = th[0];
        S->otsu_bin = ts;
        S->proxy_thr = ts;
        const long long c = ((long long)(ts + 1) * S->K + 255) / 256;
        S->q_thr = (int32_t)((long long)S->qmin + c);
    }
}
__global__ __launch_bounds__(256) void k_multi_pick(DevState* S, int classes, int parts) {
    k_multi_pick_body(hw_part(), S, classes, parts);
}

hipError_t launch_threshold(const LaunchCtx& lc, DevState* S, const roix_criterion* crit) {
    if (crit->thr != ROIX_THR_MULTI_OTSU) return launch_otsu(lc, S, crit->thr == ROIX_THR_FIXED);
    const int classes = crit->classes == 4 ? 4 : 3;
    static_assert(kMoPairBlocks * 256 >= 254 * 255 + 255, "the grid covers every pair (t1, t2)");
    static_assert(kMoChunks * kMoChunk >= 255, "the chunks cover every t3");
    const int parts = classes == 4 ? kMoParts : kMoPairBlocks;
    timer_begin(lc.timer, ST_OTSU, lc.stream);
    launch_k<256, k_multi_search_body>(lc, k_multi_search, dim3(parts), dim3(256), 0, S, classes);
    launch_k<256, k_multi_pick_body>(lc, k_multi_pick, dim3(1), dim3(256), 0, S, classes, parts);
    timer_end(lc.timer, ST_OTSU, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
