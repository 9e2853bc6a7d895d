// host.h - host-side pieces shared by the library's translation units: the
// context, the scratch-arena layout, argument checks and the launch
// sequences that the plain, batched and streamed forms have in common.
#pragma once

#include <memory>
#include <vector>

#include "common.h"

namespace roix {

struct Timer {
    bool on = false;
    struct Open {
        hipEvent_t a = nullptr;
    } open[ST_COUNT];
    struct Pending {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

}  // namespace roix

// The batched form's cached graph: the launch sequence of the last batch,
// keyed by its structure (bodies, grids, table offsets), not by its buffers.
struct BatchState {
    hipStream_t origin = nullptr;  // the graph is captured and launched here
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    uint8_t* pinned = nullptr;       // the argument tables, copied to the device from here
    size_t pinned_cap = 0, pinned_bytes = 0;
    hipEvent_t ev_copy = nullptr;    // that copy has read `pinned`
    // the last batch's merged launches, kept while its descriptors and the
    // context's parameters stay the same (then the tables are too)
    std::shared_ptr<struct BatchPlan> plan;
    std::vector<uint8_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // lanes after the first run on these streams, joined back by the events
    hipStream_t lane_stream[3] = {nullptr, nullptr, nullptr};
    hipEvent_t lane_done[3] = {nullptr, nullptr, nullptr};
};
void batch_destroy(BatchState& b);

struct roix_ctx {
    int device = 0;
    int cus = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    roix::Timer timer;
    int grid_stream = 2048;
    int grid_emit = 1536;  // workgroups of the code-emit kernels
    int grid_mask = 8192;  // workgroups of the mask-word and run kernels
    int grid_read = 512;
    int seg_grid = 512;
    int seg_runs = 0;
    int stats_grid = 512;
    uint64_t p16_min = 1ull << 22;  // fused16_min_voxels
    int batch_group = 0;  // volumes per launch group of a batch (0: as many as the arena holds)
    int batch_lanes = 2;  // concurrent launch sequences of a batch (volumes dealt out in turn)
    // smallest float32 volume a batch quantises in one pass: below this the
    // per-workgroup class tables of that pass cost more than a second read
    uint64_t batch_p16_min = 1ull << 26;
    int batch_graph = 0;  // 1: replay batches as a HIP graph (slower to launch than the ~70 direct launches here)
    BatchState batch;
};

namespace roix {

constexpr uint64_t kRunBytes = 21;  // xs, xe, parent, comp id, row (4 B each) + kept flag (1 B)

size_t align256(size_t x);
// dims -> geometry; false when a dim is < 1 or a bound of the path is exceeded
// (N <= 2^33 voxels, ny * nz < 2^31 rows, nx < 2^31 - 64)
bool geom_of(roix_dims d, Geom* g);
// largest possible number of runs: half the voxels of every row, capped
uint64_t worst_runs(const Geom& g);
// Proxy kinds of a layout: 0 none, 1 the 1-byte proxy, 2 room for the 16-bit
// proxy and the code-class tables of the fused pass (which falls back to the
// 1-byte proxy in the same buffer when the codes span more than 2^15 values).
// Kind 2 serves float32 volumes of at least kP16MinVoxels voxels whose rows
// hold a multiple of 4 voxels.
constexpr uint64_t kP16MinVoxels = 1ull << 22;
int proxy_kind(const Geom& g, roix_dtype dt, uint64_t min_voxels = kP16MinVoxels);
// bytes of the per-voxel and per-row part of a layout
// mask_rows: rows of the bitmask (-1: every row; a streamed volume kept as
// row extents holds only its staged slab's rows)
size_t fixed_bytes(const Geom& g, int proxy = 1, int64_t mask_rows = -1);
// the kind a region of `bytes` takes: kind 2 only when it still leaves room
// for the worst-case run arrays
int proxy_kind_for(const Geom& g, roix_dtype dt, size_t bytes, uint64_t min_voxels = kP16MinVoxels);
// carve a layout from [base, base + bytes); the run arrays take what is left
// (at most worst_runs); false when not even one run fits
bool carve_at(void* base, size_t bytes, const Geom& g, Layout* L, int proxy = 1, int64_t mask_rows = -1);
LaunchCtx lctx(roix_ctx* c, void* stream);
bool aligned(const void* p, size_t a);
bool eb_ok(roix_eb eb);
bool crit_ok(const roix_criterion* c);
bool out_ok(const roix_fused_out* o, bool need_comps);

// flatten -> component ids -> stats -> keep
hipError_t components_and_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, const roix_criterion* crit,
                               roix_component* comps, int64_t comps_cap);
// span scan -> codes -> row table -> outliers
hipError_t spans_and_emit(const LaunchCtx& lc, const Geom& g, const Layout& L, const void* in, roix_dtype dt,
                          const roix_fused_out* out, const BgRef* bg = nullptr);
// the whole fused path on a carved layout
roix_status enqueue_fused(const LaunchCtx& lc, const Geom& g, Layout L, const void* d_in, roix_dtype dtype,
                          roix_eb eb, const roix_criterion* crit, const roix_fused_out* out);
// the same on M = I - B, the subtraction folded into the passes that read I
roix_status enqueue_fused_bg(const LaunchCtx& lc, const Geom& g, Layout L, const float* d_in, const BgRef& bg,
                             roix_eb eb, const roix_criterion* crit, const roix_fused_out* out);

}  // namespace roix

#define ROIX_TRY(x)                                   \
    do {                                              \
        hipError_t _e = (x);                          \
        if (_e != hipSuccess) return ROIX_EDEVICE;    \
    } while (0)
