// k_background.hip - background subtraction (Sec. 4.1.1): M = I - B voxel by
// voxel, with B one calibration plane (ny x nx) for every z or a whole
// reference volume; and the inverse, I' = M' + B, that puts a decoded volume
// back on its background (the last step of the reverse process, Sec. 4.3).
//
// Both are one float32 operation per voxel (one rounding), so the result is
// exact to the last bit against any IEEE implementation.  The work is split
// into units of kBgUnit elements inside one plane: a unit's plane index is
// one division, and the reference plane's offset follows from it, so the
// per-element loop has no division.  Each lane keeps 4 loads of the input and
// 4 of the reference in flight.  The input and output are streamed
// (non-temporal); a reference plane is read with ordinary loads so that it
// stays in the caches across the z-planes.
#include "common.h"

namespace roix {

constexpr int kBgPerLane = 4;
constexpr int64_t kBgUnit = (int64_t)kBlock * kBgPerLane;  // elements (VEC: 4-voxel vectors) per unit

typedef float v4f32_t __attribute__((ext_vector_type(4)));

template <int OP>
__device__ __forceinline__ float bg_apply(float x, float b) {
    return OP == ROIX_BG_SUBTRACT ? x - b : x + b;
}

template <typename T>
__device__ __forceinline__ v4f32_t bg_load4(const T* in, int64_t i);

template <>
__device__ __forceinline__ v4f32_t bg_load4<float>(const float* in, int64_t i) {
    return __builtin_nontemporal_load(reinterpret_cast<const v4f32_t*>(in) + i);
}

template <>
__device__ __forceinline__ v4f32_t bg_load4<uint16_t>(const uint16_t* in, int64_t i) {
    const v2u32_t r = __builtin_nontemporal_load(reinterpret_cast<const v2u32_t*>(in) + i);
    v4f32_t f;
    f.x = (float)(r.x & 0xFFFFu);
    f.y = (float)(r.x >> 16);
    f.z = (float)(r.y & 0xFFFFu);
    f.w = (float)(r.y >> 16);
    return f;
}

// VEC: elements are 4-voxel vectors (plane % 4 == 0, buffers aligned);
// otherwise single voxels.  plane_e: elements per plane; full: the reference
// has a plane per z.  out may be in (float32 in place): every element is
// read and then written by the same lane.
// WHEN (the fused path's on-demand M, read from the device state S): 0
// always; 1 only when the range pass fell back to the 1-byte proxy; 2 only
// when the 16-bit proxy path queued chunks for the general emit kernel.
template <typename T, int OP, bool VEC, int WHEN = 0>
__global__ __launch_bounds__(kBlock) void k_background(const T* in, const float* __restrict__ bg, float* out,
                                                       int64_t plane_e, int64_t nz, int full,
                                                       const DevState* S) {
    if constexpr (WHEN == 1) {
        if (S->p16) return;
    } else if constexpr (WHEN == 2) {
        if (!S->p16 || S->n_slow == 0u) return;
    }
    const int64_t upp = (plane_e + kBgUnit - 1) / kBgUnit;  // units per plane
    const int64_t units = upp * nz;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t z = u / upp;
        const int64_t e0 = (u - z * upp) * kBgUnit + threadIdx.x;  // element within the plane
        const int64_t base = z * plane_e;
        const int64_t bbase = full ? base : 0;
        if (VEC) {
            v4f32_t x[kBgPerLane], b[kBgPerLane];
#pragma unroll
            for (int k = 0; k < kBgPerLane; ++k) {
                const int64_t e = e0 + (int64_t)k * kBlock;
                const int64_t es = e < plane_e ? e : 0;  // a safe address for lanes past the plane
                x[k] = bg_load4<T>(in, base + es);
                b[k] = full ? __builtin_nontemporal_load(reinterpret_cast<const v4f32_t*>(bg) + bbase + es)
                            : reinterpret_cast<const v4f32_t*>(bg)[es];
            }
#pragma unroll
            for (int k = 0; k < kBgPerLane; ++k) {
                const int64_t e = e0 + (int64_t)k * kBlock;
                if (e >= plane_e) continue;
                v4f32_t y;
                y.x = bg_apply<OP>(x[k].x, b[k].x);
                y.y = bg_apply<OP>(x[k].y, b[k].y);
                y.z = bg_apply<OP>(x[k].z, b[k].z);
                y.w = bg_apply<OP>(x[k].w, b[k].w);
                __builtin_nontemporal_store(y, reinterpret_cast<v4f32_t*>(out) + base + e);
            }
        } else {
            float x[kBgPerLane], b[kBgPerLane];
#pragma unroll
            for (int k = 0; k < kBgPerLane; ++k) {
                const int64_t e = e0 + (int64_t)k * kBlock;
                const int64_t es = e < plane_e ? e : 0;
                x[k] = (float)ld_stream(in + base + es);
                b[k] = bg[bbase + es];
            }
#pragma unroll
            for (int k = 0; k < kBgPerLane; ++k) {
                const int64_t e = e0 + (int64_t)k * kBlock;
                if (e < plane_e) __builtin_nontemporal_store(bg_apply<OP>(x[k], b[k]), out + base + e);
            }
        }
    }
}

template <typename T, int OP>
static void bg_launch(const LaunchCtx& lc, const T* in, const float* bg, float* out, const Geom& g, bool full,
                      bool vec) {
    const int64_t plane = g.nx * g.ny;
    const int64_t plane_e = vec ? plane / 4 : plane;
    const int64_t units = (plane_e + kBgUnit - 1) / kBgUnit * g.nz;
    const int grid = (int)(units < (int64_t)lc.grid_stream ? units : (int64_t)lc.grid_stream);
    if (vec)
        hipLaunchKernelGGL((k_background<T, OP, true>), dim3(grid), dim3(kBlock), 0, lc.stream, in, bg, out,
                           plane_e, g.nz, full ? 1 : 0, (const DevState*)nullptr);
    else
        hipLaunchKernelGGL((k_background<T, OP, false>), dim3(grid), dim3(kBlock), 0, lc.stream, in, bg, out,
                           plane_e, g.nz, full ? 1 : 0, (const DevState*)nullptr);
}

hipError_t launch_background(const LaunchCtx& lc, const void* in, roix_dtype dt, const float* bg, bool full,
                             const Geom& g, int op, float* out) {
    const size_t es = dt == ROIX_F32 ? 4 : 2;
    const bool vec = (g.nx * g.ny) % 4 == 0 && (uintptr_t)in % (4 * es) == 0 && (uintptr_t)bg % 16 == 0 &&
                     (uintptr_t)out % 16 == 0;
    timer_begin(lc.timer, ST_BACKGROUND, lc.stream);
    if (dt == ROIX_F32) {
        if (op == ROIX_BG_SUBTRACT)
            bg_launch<float, ROIX_BG_SUBTRACT>(lc, (const float*)in, bg, out, g, full, vec);
        else
            bg_launch<float, ROIX_BG_ADD>(lc, (const float*)in, bg, out, g, full, vec);
    } else {
        bg_launch<uint16_t, ROIX_BG_SUBTRACT>(lc, (const uint16_t*)in, bg, out, g, full, vec);
    }
    timer_end(lc.timer, ST_BACKGROUND, lc.stream);
    return hipGetLastError();
}

hipError_t launch_background_if(const LaunchCtx& lc, const float* in, const BgRef& bg, const Geom& g, DevState* S,
                                int when) {
    // the fused path with a background runs on 16-byte aligned rows of whole 64-voxel words
    const int64_t plane_e = g.nx * g.ny / 4;
    const int64_t units = (plane_e + kBgUnit - 1) / kBgUnit * g.nz;
    const int grid = (int)(units < (int64_t)lc.grid_stream ? units : (int64_t)lc.grid_stream);
    const int full = bg.plane ? 0 : 1;
    timer_begin(lc.timer, ST_BACKGROUND, lc.stream);
    if (when == 1)
        hipLaunchKernelGGL((k_background<float, ROIX_BG_SUBTRACT, true, 1>), dim3(grid), dim3(kBlock), 0, lc.stream,
                           in, bg.bg, bg.work, plane_e, g.nz, full, (const DevState*)S);
    else
        hipLaunchKernelGGL((k_background<float, ROIX_BG_SUBTRACT, true, 2>), dim3(grid), dim3(kBlock), 0, lc.stream,
                           in, bg.bg, bg.work, plane_e, g.nz, full, (const DevState*)S);
    timer_end(lc.timer, ST_BACKGROUND, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
