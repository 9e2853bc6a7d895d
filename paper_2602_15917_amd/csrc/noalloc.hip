// noalloc.hip - roix_fused_noalloc: the fused path on a fixed-size scratch
// array compiled into the library, for callers that may not allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The kernels and the launch sequence are those of
// roix_fused; only the arena differs.
#include <mutex>

#include "host.h"

using namespace roix;

namespace {

// The arena of every call on one device: file-scope device memory, one copy
// per GPU, held until the process ends.  In host code this name is only a
// stand-in for the symbol; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[ROIX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceArena {
    void* ptr = nullptr;  // device address of `scratch` on this device
    int cus = 0;
    hipError_t err = hipSuccess;
    std::once_flag once;
};

DeviceArena g_arena[kMaxDevices];

// once per device, with that device current: resolve the array's address
// and the compute-unit count the launch grids are sized from
void arena_setup(DeviceArena& a, int dev) {
    void* p = nullptr;
    a.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (a.err != hipSuccess) return;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    a.cus = cus;
    a.ptr = p;
}

}  // namespace

extern "C" roix_status roix_fused_noalloc(const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                                          const roix_criterion* crit, const roix_fused_out* out, void* stream) {
    Geom g;
    if (!d_in || !geom_of(dims, &g) || !eb_ok(eb) || !crit_ok(crit) || !out_ok(out, true)) return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (!aligned(d_in, dtype == ROIX_F32 ? 4 : 2)) return ROIX_EINVAL;
    // the worst-case layout of the volume must fit the array: then no run
    // capacity or proxy choice can depend on the data
    const size_t need = fixed_bytes(g, proxy_kind(g, dtype)) + (size_t)worst_runs(g) * kRunBytes;
    if (need > (size_t)ROIX_NOALLOC_SCRATCH_BYTES) return ROIX_ENOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ROIX_EDEVICE;
    DeviceArena& a = g_arena[dev];
    std::call_once(a.once, arena_setup, std::ref(a), dev);
    if (a.err != hipSuccess || !a.ptr) return ROIX_EDEVICE;
    const size_t bytes = (size_t)ROIX_NOALLOC_SCRATCH_BYTES;
    Layout L;
    if (!carve_at(a.ptr, bytes, g, &L, proxy_kind_for(g, dtype, bytes))) return ROIX_ENOMEM;
    // the default launch parameters of a new context on this device
    LaunchCtx lc;
    lc.stream = (hipStream_t)stream;
    lc.timer = nullptr;
    lc.grid_stream = a.cus * 8;
    lc.grid_read = a.cus * 4;
    lc.grid_emit = a.cus * 6;
    lc.grid_mask = a.cus * 32;
    lc.seg_grid = a.cus * 2;
    lc.seg_runs = 0;
    lc.stats_grid = a.cus;
    return enqueue_fused(lc, g, L, d_in, dtype, eb, crit, out);
}
