// common.h - device state, scratch layout and launcher declarations shared by
// the HIP translation units of libroix.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <utility>
#include <vector>

#include "../../include/roix.h"

namespace roix {

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kHistCopies = 32;      // LDS-privatised histogram copies (one per half-wave lane)
constexpr int kHistStride = 257;     // copy stride: lane c + bin b lands in bank (c + b) mod 32
constexpr int kScanBlocks = 1024;    // fixed block count of the device-sized scans
// MI355X's last-level (Infinity) cache, shared by the XCDs
constexpr int64_t kLastLevelCache = 256ll << 20;
constexpr int kKeepGrid = 512;       // workgroups of the keep rule
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kQrFine = 1 << 15;  // code classes (q mod 2^15) of the fused 16-bit proxy pass
constexpr int kQrBlocks = 256;    // workgroups of that pass (one LDS class table each)
constexpr int kMoPairBlocks = 256; // multi-level Otsu search: workgroups over the pairs (t1, t2)
constexpr int kMoChunks = 8;       // K = 4: t3 ranges of kMoChunk thresholds per pair
constexpr int kMoChunk = 32;
constexpr int kMoParts = kMoPairBlocks * kMoChunks;  // partial results of the search
constexpr int kEmitSlice = 256;  // codes per emit slice: 4 consecutive codes per lane
constexpr int kEmitSlices = 4;   // slices per emit step (16-byte loads in flight per lane)
constexpr int kEmitSteps = 4;
constexpr uint64_t kEmitChunk = (uint64_t)kEmitSlice * kEmitSlices * kEmitSteps;  // codes per emit work item

// Everything the kernels of one call share, reset by k_init at the start of
// the call (no memset: the sequence can be captured into a graph).
struct DevState {
    int32_t status;   // first fatal data error (ROIX_EINVAL/ERANGE/ENOMEM/ETRUNC/EDEVICE)
    int32_t trunc;    // an output buffer was too small (counts still complete)
    int32_t qstatus;  // error of the quantiser resolution alone
    int32_t pad3;
    uint32_t kmin, kmax;
    uint32_t nonfinite;
    uint32_t pad0;
    // resolved quantiser
    float xmin, xmax, eb32, w, r, binscale;
    int32_t qmin, qmax, width_bits;
    uint32_t esc;
    int64_t K;
    uint32_t bin_mlo, bin_mhi;  // ceil(2^40 / K): bin = umulhi(u, mlo) + u * mhi when K <= 65536
    uint32_t bin_a, bin_m24;    // K <= 46340: bin = ((u << a) * m24) >> 32 on 24-bit operands (m24 0: none)
    // threshold
    int32_t otsu_bin, q_thr, proxy_thr;
    uint32_t flags;
    unsigned long long hist[256];
    unsigned long long n_mask;
    // labelling
    uint32_t n_runs, n_comps;
    unsigned long long max_size;
    uint32_t largest_cid, pad1;
    uint32_t bbox[6];
    unsigned long long n_kept, n_kept_voxels;
    // extraction
    unsigned long long span_total;  // (rows with a span) << 40 | (codes)
    unsigned long long n_outliers, q_outliers;
    uint32_t n_slow;  // emit chunks queued for the general chunk kernel
    uint32_t p16;     // the proxy is the 16-bit code proxy (fused pass, K <= 2^15)
    // run number where the current labelling pass starts (0 for a whole
    // volume; the first run of the slab for a streamed slab)
    uint32_t seg_lo;
    // streamed volumes: the mask parameters fixed at open (r, and rint(T r)
    // of the fixed threshold), and the status held back over the close
    // sequence's quantiser stages
    int32_t saved_status;
    float serve_r, serve_rt;
    // streamed volumes kept as row extents: values of the store in use, and
    // the extent total of the slab being stored
    unsigned long long store_used, store_slab;
    // threshold search: the thresholds and class count, and the multi-level
    // Otsu search's best (score, tuple rank) per workgroup
    int32_t thr_t[3];
    int32_t n_classes;
    double mo_val[kMoParts];
    unsigned long long mo_rank[kMoParts];
    // LARGEST: the keep workgroups done, and each one's largest size and the
    // first component holding it
    uint32_t done_keep, pad2;
    // LARGEST: the kept component's root run (kNone: none), for passes that
    // test a run's root instead of looking up its component's kept flag
    uint32_t kept_root, kept_by_root;
    unsigned long long keep_size[kKeepGrid];
    uint32_t keep_cid[kKeepGrid];
};

// Per-call view of the scratch arena.
struct Layout {
    DevState* S;
    uint8_t* proxy;         // nrows * W * 64 bytes, or twice that for the 16-bit proxy (see Geom)
    uint64_t* maskbits;     // nrows * W words
    uint32_t* row_nruns;    // nrows
    uint32_t* run_off;      // nrows + 1
    uint32_t* run_xs;       // run_cap
    uint32_t* run_xe;       // run_cap
    uint32_t* parent;       // run_cap
    uint32_t* comp_id;      // run_cap (root flags, then component ids)
    uint32_t* run_row;      // run_cap (row z * ny + y of each run)
    uint8_t* kept_flag;     // run_cap (per component)
    uint32_t* row_xs;       // nrows
    uint32_t* row_xe;       // nrows
    uint64_t* row_packed;   // nrows (has_span << 40 | span length), scanned in place
    uint64_t* row_outl;     // nrows: outliers per row, then their exclusive scan
    uint32_t* nz_rows;      // nrows: row of the i-th span
    uint64_t* span_desc;    // 2 * nrows: per span, its first code and voxel - code offset
    uint32_t* chunk_row;    // N / kEmitChunk + 2: span holding the first code of each emit chunk
    uint32_t* slow_chunks;  // N / kEmitChunk + 2: chunks left to the general chunk kernel
    uint64_t* scan_tmp;     // kScanBlocks + 1
    int32_t* slice_thr;     // nz: threshold bin of each slice (per-slice Otsu)
    uint32_t* fine_slots;   // kQrBlocks * kQrFine, or null (no 16-bit proxy)
    unsigned long long* fine_total;  // kQrFine
    uint64_t run_cap;
    // Where the input values of row r start: element row_org[r] of the value
    // array is voxel (r, x = 0), so voxel (r, x) is element row_org[r] + x.
    // Null: the volume itself, row_org = r * nx.  A streamed volume that keeps
    // only each row's extent sets this (values outside the extent are never
    // read).  nvals: elements of the value array (0: the N voxels).
    const uint64_t* row_org;
    uint64_t nvals;
};

__device__ __forceinline__ uint64_t row_origin(const Layout& L, uint32_t rid, int64_t nx) {
    return L.row_org ? L.row_org[rid] : (uint64_t)rid * (uint64_t)nx;
}

// The proxy of row r, voxel x is element r * 64 W + x (a byte, or a 16-bit
// word for the 16-bit proxy): rows are padded to whole 64-voxel words, so one
// lane can turn 64 proxy elements into one mask word.  Padding elements are
// never read as object: the mask of a row's last word is cut at nx.
struct Geom {
    int64_t nx, ny, nz;
    uint64_t N;
    int64_t nrows;  // ny * nz
    int64_t W;      // 64-bit words per row of the bitmask
};

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ void fail(DevState* S, int32_t st) { atomicCAS(&S->status, 0, st); }

__device__ __forceinline__ uint32_t f2key(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(b);
}

// code of a value: fp32 multiply (no contraction: built with -ffp-contract=off),
// round to nearest even.  The rounded value is clamped into int32 range
// before the conversion (maxNum/minNum: a NaN becomes the lower bound), so the
// conversion is defined for every input; codes with |x r| > 2^24 or of a
// non-finite voxel are never used (ERANGE, EINVAL), and inside that range the
// clamp changes nothing.
__device__ __forceinline__ int32_t qcode(float x, float r) {
    const float t = __builtin_rintf(x * r);
    return (int32_t)__builtin_fminf(__builtin_fmaxf(t, -2147483648.0f), 2147483520.0f);
}

__device__ __forceinline__ bool outlier(float x, int32_t q, float w, float eb32) {
    float xh = (float)q * w;
    float d = x - xh;
    return !(__builtin_fabsf(d) <= eb32);
}

// exact bin = floor(256 u / K) for 0 <= u < K <= 2^25 + 1: a float estimate,
// off by at most one near a bin edge, then one integer correction.
__device__ __forceinline__ uint32_t bin_slow(uint32_t u, uint32_t K, float binscale) {
    uint32_t t = (uint32_t)((float)u * binscale);
    t = t > 255u ? 255u : t;
    uint64_t u256 = (uint64_t)u << 8;
    if ((uint64_t)t * K > u256) t -= 1u;
    else if ((uint64_t)(t + 1u) * K <= u256) t += 1u;
    return t;
}

// exact bin for K <= 65536 with M = ceil(2^40 / K): (u * M) >> 32 equals
// floor(256 u / K) because the rounding excess u (M - 2^40/K) / 2^32 stays
// below 1/K when K (K - 1) <= 2^32 (checked exhaustively for every K and u).
__device__ __forceinline__ uint32_t bin_fast(uint32_t u, uint32_t mlo, uint32_t mhi) {
    return __umulhi(u, mlo) + u * mhi;
}

// exact bin for K <= 46340 with 24-bit operands (one full-rate multiply-high):
// a and m = ceil(2^(40-a) / K) are chosen so that m < 2^24, (K - 1) 2^a <
// 2^24 and K^2 2^a <= 2^32; the excess of ((u 2^a) m) / 2^32 over 256 u / K
// is then below 1/K, so the floor is exact (checked exhaustively for every
// K <= 46340 and u < K).
__device__ __forceinline__ uint32_t bin24(uint32_t u, uint32_t a, uint32_t m) {
    return (uint32_t)(((uint64_t)((u << a) & 0xFFFFFFu) * (uint64_t)(m & 0xFFFFFFu)) >> 32);
}
// a and m of bin24 for K (the smallest a with m < 2^24); m = 0: no such form
__device__ __forceinline__ void bin24_params(uint64_t K, uint32_t& a, uint32_t& m) {
    a = 0u;
    m = 0u;
    if (K < 1 || K > 46340) return;
    for (uint32_t t = 0; t <= 24; ++t) {
        const uint64_t mt = ((1ull << (40 - t)) + K - 1ull) / K;
        if (mt >= (1ull << 24)) continue;
        if (K * K * (1ull << t) <= (1ull << 32) && ((K - 1ull) << t) < (1ull << 24)) {
            a = t;
            m = (uint32_t)mt;
        }
        return;
    }
}

// Non-temporal loads for data streamed once (the volume): they do not
// displace the reused run tables from the caches.
typedef unsigned int v4u32_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const v4u32_t v = __builtin_nontemporal_load(reinterpret_cast<const v4u32_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ uint16_t ld_stream(const uint16_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t ld_stream(const int32_t* p) { return __builtin_nontemporal_load(p); }
typedef unsigned int v2u32_t __attribute__((ext_vector_type(2)));
typedef unsigned int v3u32_t __attribute__((ext_vector_type(3)));
__device__ __forceinline__ void st_stream(uint2* p, uint2 v) {
    v2u32_t t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2u32_t*>(p));
}

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hand-offs between the workgroups of one launch use no cache maintenance
// (a device-scope fence writes back and invalidates a whole L2 on this
// chip, and costs tens of microseconds when every workgroup issues one).
// Instead the words handed over are written and read only with device-scope
// atomic accesses, which are coherent across the XCDs' L2s, and a wave that
// signals first waits for its own memory operations to complete; the signal
// fences keep the compiler from moving memory accesses across the wait.
__device__ __forceinline__ void wait_mem() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS written by some lanes of a wave is read by others after this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves by DPP (a VALU operand modifier, no LDS traffic).  Lane i
// reads lane i + n (row_shl n) or i - n (row_shr n) of its row of 16 lanes,
// the lane given by a quad pattern of its group of 4, lane 15 (31) broadcast
// to the rows after it, or lane i - 1 of the wave (wave_shr 1).  A lane whose
// source lies outside its row or wave, or whose row is not in ROWS, gets `old`.
constexpr int kDppRowShl = 0x100, kDppRowShr = 0x110, kDppWaveShr1 = 0x138, kDppBcast15 = 0x142,
              kDppBcast31 = 0x143, kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E;
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

// Inclusive prefix sum over the 64 lanes: shifts 1, 2, 4, 8 inside each row
// of 16, then the total of row 0 added to row 1 and of row 2 to row 3, then
// that of rows 0-1 to rows 2-3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_u32<kDppRowShr + 1>(0u, v);
    v += dpp_u32<kDppRowShr + 2>(0u, v);
    v += dpp_u32<kDppRowShr + 4>(0u, v);
    v += dpp_u32<kDppRowShr + 8>(0u, v);
    v += dpp_u32<kDppBcast15, 0xA>(0u, v);
    v += dpp_u32<kDppBcast31, 0xC>(0u, v);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

// ------------------------------------------------------------ stage timing

enum Stage {
    ST_INIT = 0,
    ST_RANGE,
    ST_RESOLVE,
    ST_QUANTIZE,
    ST_HIST,
    ST_QR16,
    ST_OTSU,
    ST_MASK_RUNS,
    ST_SCAN,
    ST_RUNS,
    ST_UNION,
    ST_FLATTEN,
    ST_COMPS,
    ST_KEEP,
    ST_SPANS,
    ST_EMIT,
    ST_EMIT_ROWS,
    ST_VOXEL_OUT,
    ST_FINALIZE,
    ST_DECODE_INDEX,
    ST_DECODE,
    ST_BACKGROUND,
    ST_ABSQ,
    ST_HUFF,
    ST_SECTION,
    ST_COUNT
};

struct Timer;  // defined in api.hip
void timer_begin(Timer* t, int stage, hipStream_t s);
void timer_end(Timer* t, int stage, hipStream_t s);

// ------------------------------------------------- one launch, many volumes
//
// Every kernel of the fused path is a body run on a virtual grid: VPart.b is
// the workgroup's index among the VPart.n workgroups that work on one
// volume.  A plain launch gives the body the hardware grid.  A batch records
// each volume's launches (body, grid, arguments) instead of launching them,
// then launches each body once for all the volumes that need it next: the
// arguments of every volume in a device table, and the workgroups split by
// a prefix table of the volumes' grids (a workgroup finds its volume by
// binary search).  Each volume sees exactly the grid and arguments of its
// plain launch, and its launches keep their order.

struct VPart {
    uint32_t b, n;
};

__device__ __forceinline__ VPart hw_part() { return VPart{blockIdx.x, gridDim.x}; }

template <class... A>
struct ArgPack;
template <>
struct ArgPack<> {};
template <class H, class... T>
struct ArgPack<H, T...> {
    H h;
    ArgPack<T...> t;
};

inline ArgPack<> make_pack() { return ArgPack<>{}; }
template <class H, class... T>
inline ArgPack<H, T...> make_pack(H h, T... t) {
    return ArgPack<H, T...>{h, make_pack(t...)};
}

template <size_t I, class H, class... T>
__host__ __device__ __forceinline__ const auto& pack_get(const ArgPack<H, T...>& p) {
    if constexpr (I == 0)
        return p.h;
    else
        return pack_get<I - 1>(p.t);
}

template <auto Body, class... A, size_t... I>
__device__ __forceinline__ void pack_call(VPart vp, const ArgPack<A...>& p, std::index_sequence<I...>) {
    Body(vp, pack_get<I>(p)...);
}

// start[v] = first workgroup of volume v, start[n] = the grid, start[n + 1]
// = kTableMark: a table that did not arrive intact runs nothing
constexpr uint32_t kTableMark = 0x5849'4F52u;
template <int LB, auto Body, class... A>
__global__ __launch_bounds__(LB) void k_many(const ArgPack<A...>* __restrict__ args,
                                             const uint32_t* __restrict__ start, uint32_t n) {
    if (start[n + 1] != kTableMark) return;  // uniform
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    const uint32_t s0 = start[lo];
    pack_call<Body>(VPart{b - s0, start[lo + 1] - s0}, args[lo], std::index_sequence_for<A...>{});
}

using ManyLaunch = void (*)(const void* args, const uint32_t* start, uint32_t n, uint32_t grid, uint32_t block,
                            uint32_t shmem, hipStream_t s);

template <int LB, auto Body, class... A>
void many_launch(const void* args, const uint32_t* start, uint32_t n, uint32_t grid, uint32_t block, uint32_t shmem,
                 hipStream_t s) {
    hipLaunchKernelGGL((k_many<LB, Body, A...>), dim3(grid), dim3(block), shmem, s,
                       reinterpret_cast<const ArgPack<A...>*>(args), start, n);
}

// One recorded launch of one volume.
struct RecLaunch {
    ManyLaunch launch;  // also the key: one per (body, block bound, argument types)
    uint32_t grid, block, shmem;
    uint32_t arg_size, arg_align;
    std::vector<uint8_t> args;
};

struct Recorder {
    std::vector<RecLaunch> seq;
    bool bad = false;  // a launch that cannot be recorded (a 2-D grid)
    template <int LB, auto Body, class... A>
    void add(dim3 grid, dim3 block, size_t shmem, const ArgPack<A...>& p) {
        if (grid.y != 1 || grid.z != 1 || block.y != 1 || block.z != 1) bad = true;
        RecLaunch r;
        r.launch = &many_launch<LB, Body, A...>;
        r.grid = grid.x;
        r.block = block.x;
        r.shmem = (uint32_t)shmem;
        r.arg_size = (uint32_t)sizeof(ArgPack<A...>);
        r.arg_align = (uint32_t)alignof(ArgPack<A...>);
        r.args.resize(sizeof(ArgPack<A...>));
        memcpy(r.args.data(), &p, sizeof(ArgPack<A...>));
        seq.push_back(std::move(r));
    }
};

struct LaunchCtx {
    hipStream_t stream;
    Timer* timer;  // may be null
    int grid_stream;  // workgroups of the grid-stride streaming kernels
    int grid_read;    // workgroups of the read-only streaming kernel (range)
    int grid_emit;    // workgroups of the code-emit kernels
    int grid_mask;    // workgroups of the mask-word and run kernels
    int seg_grid;     // workgroups of the segment labelling kernels
    int seg_runs;     // runs per segment (0: spread the runs over seg_grid)
    int stats_grid;   // workgroups of the component statistics kernel
    int scan_grid = kScanBlocks;  // chunks of the device-sized scans (at most kScanBlocks)
    int grid_vox = 0;             // quantise + histogram pass (0: grid_stream); a batch scales it
    Recorder* rec = nullptr;      // batch: record the launches instead of making them
    int cus = 0;                  // compute units of the device (0: unknown)
};

// Launch kernel `kern` (whose body is Body, block bound LB), or record it.
template <int LB, auto Body, class K, class... A>
inline void launch_k(const LaunchCtx& lc, K kern, dim3 grid, dim3 block, size_t shmem, A... a) {
    if (lc.rec)
        lc.rec->add<LB, Body>(grid, block, shmem, make_pack(a...));
    else
        hipLaunchKernelGGL(kern, grid, block, shmem, lc.stream, a...);
}

// ------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.

// eb_abs > 0: the quantiser of this absolute bound is set up too (fused pass)
hipError_t launch_init(const LaunchCtx& lc, DevState* S, double eb_abs = 0.0);
hipError_t launch_range(const LaunchCtx& lc, const void* in, roix_dtype dt, uint64_t N, DevState* S);
hipError_t launch_resolve_dt(const LaunchCtx& lc, DevState* S, roix_dtype dt, roix_eb eb,
                             const roix_criterion* crit);
hipError_t launch_seg_init(const LaunchCtx& lc, DevState* S, const roix_quant_info* qinfo,
                           const roix_criterion* crit);
hipError_t launch_quantize(const LaunchCtx& lc, const void* in, roix_dtype dt, uint64_t N, DevState* S,
                           int32_t* codes, uint32_t* outlier_bits);
// src_kind: 0 = f32 values, 1 = u16 values, 2 = int32 codes
hipError_t launch_quant_hist(const LaunchCtx& lc, const void* in, int src_kind, const Geom& g, DevState* S,
                             uint8_t* proxy, bool fixed, bool unless_p16 = false);
// float32, absolute bound, rows 16-byte aligned and a multiple of 4 voxels:
// range keys, 16-bit proxy and code-class counts in one pass; then the
// quantiser and (K <= 2^15) the histogram, setting S->p16
// A background reference subtracted on the fly (M = I - B): bg holds one
// ny x nx plane (plane = true: row r reads plane row r % ny) or a plane per
// z; work (N floats) receives M where a stage must read M itself.
struct BgRef {
    const float* bg;
    bool plane;
    float* work;
};
hipError_t launch_quant_range16(const LaunchCtx& lc, const float* in, const Geom& g, const Layout& L,
                                const BgRef* bg = nullptr);
hipError_t launch_resolve16(const LaunchCtx& lc, const Layout& L, roix_eb eb, const roix_criterion* crit);
hipError_t launch_otsu(const LaunchCtx& lc, DevState* S, bool fixed);
// the threshold of a criterion: Otsu, multi-level Otsu or fixed (whose q_thr
// the resolve step has set)
hipError_t launch_threshold(const LaunchCtx& lc, DevState* S, const roix_criterion* crit);

// u16_in: the mask from a uint16 volume whose rows are whole 64-voxel words
// (16-byte aligned) instead of the proxy
hipError_t launch_mask_runs(const LaunchCtx& lc, const Geom& g, const Layout& L, const int32_t* slice_thr = nullptr,
                            const uint16_t* u16_in = nullptr);
// streamed volumes (FIXED threshold, ABS bound): mask parameters at open,
// then per slab of rows [r0, r1) the range, mask words and run counts
hipError_t launch_serve_open(const LaunchCtx& lc, DevState* S, double eb_value, double fixed_value);
hipError_t launch_slab_mask(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g, int64_t r0,
                            int64_t r1, const Layout& L);
// the histogram of the whole volume without the proxy (streamed volumes)
hipError_t launch_hist_only(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g, DevState* S);
// Streamed uint16 volumes kept as row extents (codes within 2^15 classes):
// clear the class table and the store counters; count the code classes of a
// slab's n values; store the extent of each slab row [r0, r1) (the span of
// the row's runs) from the slab's values at `stage` into `store` (cap values),
// setting row_org; at close, resolve the quantiser and rebuild the histogram
// from the class counts
hipError_t launch_store_open(const LaunchCtx& lc, DevState* S, unsigned long long* classes);
hipError_t launch_slab_classes(const LaunchCtx& lc, const uint16_t* stage, uint64_t n, DevState* S,
                               unsigned long long* classes);
hipError_t launch_store_rows(const LaunchCtx& lc, const Geom& g, const Layout& L, const uint16_t* stage, int64_t r0,
                             int64_t r1, uint16_t* store, uint64_t cap, uint64_t* row_org, uint64_t* lens);
hipError_t launch_serve_resolve(const LaunchCtx& lc, DevState* S, double eb_value, double fixed_value,
                                const unsigned long long* classes);
// save = 1: hold back and clear the status; save = 0: restore it unless a
// newer error is set
hipError_t launch_serve_status(const LaunchCtx& lc, DevState* S, int save);
// Exclusive scans (in place allowed).  n from the host, or from *n_dev when
// n_dev is not null (then n_host is only an upper bound).  total_out and
// out_end (nullable) receive the sum of all elements.  With cap_S, a total
// above cap fails cap_S with cap_err.
// The component-id scan (ci non-null) also writes the entry of each
// component below ci->cap (its root run's first voxel as the label, size 0,
// an empty box, not kept) and clears its kept flag, unless the call has
// failed.
struct CompInit {
    const uint32_t* xs;
    const uint32_t* run_row;
    int64_t nx;
    roix_component* comps;
    uint8_t* kept_flag;
    uint64_t cap;
};
hipError_t launch_scan_u32(const LaunchCtx& lc, const uint32_t* in, uint32_t* out, int64_t n_host,
                           const uint32_t* n_dev, uint32_t* total_out, uint32_t* out_end, uint64_t* tmp,
                           DevState* cap_S = nullptr, uint64_t cap = 0, int cap_err = 0,
                           const CompInit* ci = nullptr);
hipError_t launch_scan_u64(const LaunchCtx& lc, const uint64_t* in, uint64_t* out, int64_t n_host,
                           unsigned long long* total_out, uint64_t* tmp);
// runs of rows [r0, r1); their numbers continue from run_off[r0]
hipError_t launch_runs_write(const LaunchCtx& lc, const Geom& g, const Layout& L, int64_t r0, int64_t r1);
// exclusive scan of n_host u32 counts starting from *base (device); *base
// becomes base + total, *lo_out the old base, *out_end the new total;
// tmp[kScanBlocks] receives the new 64-bit total
hipError_t launch_scan_u32_base(const LaunchCtx& lc, const uint32_t* in, uint32_t* out, int64_t n_host,
                                uint32_t* base, uint32_t* lo_out, uint32_t* out_end, uint64_t* tmp,
                                DevState* cap_S = nullptr, uint64_t cap = 0, int cap_err = 0);
hipError_t launch_union(const LaunchCtx& lc, const Geom& g, const Layout& L, int conn);
// the reverse process into out (N float32); desc: 2 * ny * nz uint4 of scratch
hipError_t launch_decode(const LaunchCtx& lc, const roix_row* rows, uint64_t rows_cap, const void* stream,
                         uint64_t stream_cap, const float* outl, uint64_t outl_cap, const roix_quant_info* qi,
                         const roix_extract_info* ei, const Geom& g, float background, float* out, DevState* S,
                         uint4* desc, roix_decode_info* dinfo);
hipError_t launch_background(const LaunchCtx& lc, const void* in, roix_dtype dt, const float* bg, bool full,
                             const Geom& g, int op, float* out);
// M = in - bg into bg.work, only when the device state asks for it:
// when = 1 after the fused range pass when it fell back to the 1-byte proxy
// (p16 == 0); when = 2 before the general emit kernel when the proxy path
// queued chunks for it (p16 == 1 and n_slow > 0)
hipError_t launch_background_if(const LaunchCtx& lc, const float* in, const BgRef& bg, const Geom& g, DevState* S,
                                int when);
hipError_t launch_slice_otsu(const LaunchCtx& lc, const Geom& g, const uint8_t* proxy, DevState* S, int32_t* thr,
                             int32_t* slice_thr_out);
size_t absq_scratch_bytes(int64_t m);
size_t huff_scratch_bytes();
hipError_t launch_huff_encode(const LaunchCtx& lc, const uint8_t* in, int64_t n, uint8_t* lengths,
                              unsigned long long* block_off, uint16_t* sub_bits, uint32_t* payload, int64_t cap_words,
                              void* scratch, roix_huff_info* info);
hipError_t launch_huff_decode(const LaunchCtx& lc, const uint8_t* lengths, const unsigned long long* block_off,
                              const uint16_t* sub_bits, const uint32_t* payload, int64_t payload_words, int64_t n,
                              uint8_t* out, void* scratch, roix_huff_info* info);
size_t section_scratch_bytes();  // the escape list's counter; the list takes the rest of the arena
hipError_t launch_section(const LaunchCtx& lc, const void* in, roix_dtype dt, const Geom& g,
                          const roix_fused_out* o, uint8_t* out, int64_t out_cap, roix_section_info* info,
                          void* scratch, size_t scratch_bytes);
hipError_t launch_absq(const LaunchCtx& lc, const uint8_t* D, int64_t m, uint32_t K, uint8_t* Q, void* scratch,
                       roix_absq_info* info);
hipError_t launch_flatten(const LaunchCtx& lc, const Geom& g, const Layout& L);
hipError_t launch_comp_stats(const LaunchCtx& lc, const Geom& g, const Layout& L, roix_component* comps);
hipError_t launch_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, roix_component* comps,
                       const roix_criterion* crit);
hipError_t launch_voxel_out(const LaunchCtx& lc, const Geom& g, const Layout& L, const roix_component* comps,
                            uint8_t* keep, int64_t* labels);

hipError_t launch_spans_from_runs(const LaunchCtx& lc, const Geom& g, const Layout& L);
hipError_t launch_spans_from_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, const uint8_t* keep);
// with bg: `in` is the image I; the codes come from the 16-bit proxy, the
// queued chunks read M from bg->work, the outlier values are I - B
hipError_t launch_emit(const LaunchCtx& lc, const Geom& g, const Layout& L, const void* in, roix_dtype dt,
                       const roix_fused_out* out, const BgRef* bg = nullptr);
// mode bits: 1 = quant info, 2 = seg info, 4 = extract info; fused marks n_outliers not computed
hipError_t launch_finalize(const LaunchCtx& lc, DevState* S, roix_quant_info* qi, roix_seg_info* si,
                           roix_extract_info* ei, bool fused_q);

}  // namespace roix
