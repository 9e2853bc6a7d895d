// serve.hip - the served form: volumes that arrive slab by slab.
//
// A server owns one HBM pool (carved first-fit per admitted volume), a copy
// stream and a compute stream.  Each slab is copied into its volume's
// resident input buffer on the copy stream; the compute stream waits for the
// copy and, for volumes whose mask is decidable per voxel (absolute bound,
// FIXED threshold), reduces the slab at once: range, mask words, runs, and
// the union of the slab's runs with the runs of the earlier slabs, all kept
// in the volume's device state.  The close runs what needs the whole volume
// (resolve, histogram, keep, spans, codes).  Other volumes run the whole
// fused path at close.  Completion times come from timing events measured
// against a reference event recorded when the server was created.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <thread>

#include <string.h>

#include "host.h"

using namespace roix;

namespace {

constexpr int64_t kServeRunsPerRow = 32;  // default run-array capacity of a served volume, per row
constexpr int64_t kSlabPlanes = 32;       // default planes staged at once by a volume kept as row extents
constexpr int64_t kStorePermille = 500;   // default store of such a volume, per mille of its voxels

// First-fit allocator over [0, size) in 256-byte units.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0, used = 0;

    void init(size_t n) {
        free_.clear();
        size = n & ~(size_t)255;
        if (size) free_[0] = size;
        used = 0;
    }
    bool alloc(size_t n, size_t* off) {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest) free_[o + n] = rest;
            *off = o;
            used += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align256(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum VolState { V_OPEN = 0, V_CLOSING = 1, V_ABORTED = 2 };

struct Vol {
    Geom g;
    roix_dtype dt;
    roix_eb eb;
    roix_criterion crit;
    roix_fused_out out;
    bool incremental = false;
    size_t off = 0, bytes = 0;  // pool region
    uint8_t* d_vol = nullptr;   // resident input (whole volumes)
    Layout L;
    int64_t next_z = 0;
    VolState state = V_OPEN;
    hipEvent_t release_ev = nullptr;  // aborted: the pool region is free once this completes
    // kept as row extents: the staged slab, the store of row extents, the
    // code-class counts and per-row tables; stage_free marks the compute of
    // the staged planes done (the next copy into the stage waits for it)
    bool compact = false;
    int64_t stage_planes = 0;
    uint16_t* stage = nullptr;
    uint16_t* store = nullptr;
    uint64_t store_cap = 0;  // values
    uint64_t* row_org = nullptr;
    uint64_t* lens = nullptr;
    unsigned long long* classes = nullptr;
    hipEvent_t stage_free = nullptr;
};

// Geometry of a volume kept as row extents, in bytes from its region start.
struct CompactPlan {
    size_t stage, store, row_org, lens, classes, layout, total;
    uint64_t store_cap;
};

struct Req {
    int64_t vol = 0;
    int kind = ROIX_REQ_SLAB;
    double submit_ms = 0.0, done_ms = 0.0;
    hipEvent_t done = nullptr;
    bool finished = false;
    int32_t status = ROIX_OK;
};

bool incremental_of(roix_eb eb, const roix_criterion* crit) {
    return eb.mode == ROIX_EB_ABS && crit->thr == ROIX_THR_FIXED;
}

// A uint16 volume with an absolute bound and a fixed threshold is kept as row
// extents when every uint16 value codes within 2^15 classes: the device's
// bound resolution (fp32 bound rounded toward zero, w = 2 eb32, r = 1 / w
// through binary64) redone here, then rint(65535 r) <= 2^15 - 1, so that
// K = qmax - qmin + 1 <= 2^15 whatever the data (the codes of 0 and 65535
// bound every code).
bool compact_of(roix_dtype dt, roix_eb eb, const roix_criterion* crit) {
    if (dt != ROIX_U16 || !incremental_of(eb, crit)) return false;
    if (!(eb.value > 0.0) || !(eb.value <= 3.4028234663852886e38)) return false;
    float eb32 = (float)eb.value;
    if ((double)eb32 > eb.value) eb32 = nextafterf(eb32, 0.0f);
    if (!std::isnormal(eb32)) return false;
    const float w = eb32 + eb32;
    const float r = (float)(1.0 / (double)w);
    if (!std::isnormal(w) || !std::isnormal(r)) return false;
    const float q = rintf(65535.0f * r);
    return q <= 32767.0f;
}

size_t runs_bytes(const Geom& g, int64_t runs_per_row) {
    uint64_t runs = (uint64_t)g.nrows * (uint64_t)runs_per_row;
    const uint64_t w = worst_runs(g);
    if (runs > w) runs = w;
    return (size_t)runs * kRunBytes;
}

CompactPlan compact_plan(const Geom& g, int64_t slab_planes, int64_t permille, int64_t runs_per_row) {
    CompactPlan p;
    const int64_t sp = slab_planes < g.nz ? slab_planes : g.nz;
    p.store_cap = (g.N * (uint64_t)permille + 999) / 1000;
    size_t o = 0;
    p.stage = o;
    o += align256((size_t)sp * (size_t)g.nx * (size_t)g.ny * 2);
    p.store = o;
    o += align256((size_t)p.store_cap * 2 + 64);
    p.row_org = o;
    o += align256((size_t)g.nrows * 8);
    p.lens = o;
    o += align256((size_t)sp * (size_t)g.ny * 8);
    p.classes = o;
    o += align256((size_t)kQrFine * 8);
    p.layout = o;
    o += fixed_bytes(g, 0, sp * g.ny) + runs_bytes(g, runs_per_row);
    p.total = o;
    return p;
}

size_t volume_bytes(const Geom& g, roix_dtype dt, bool incremental, int64_t runs_per_row, uint64_t p16_min) {
    const size_t in = align256((size_t)g.N * (dt == ROIX_F32 ? 4 : 2));
    return in + fixed_bytes(g, incremental ? 0 : proxy_kind(g, dt, p16_min)) + runs_bytes(g, runs_per_row);
}

double pct(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    const size_t k = (size_t)(p * (double)(v.size() - 1) + 0.5);
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

}  // namespace

struct roix_server {
    roix_ctx* ctx = nullptr;
    void* base = nullptr;
    Pool pool;
    hipStream_t copy = nullptr, compute = nullptr;
    hipEvent_t ev_ref = nullptr, ev_copy = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::map<int64_t, Vol> vols;
    std::map<int64_t, Req> reqs;
    std::vector<hipEvent_t> events;  // idle timing events
    int64_t next_vol = 1, next_req = 1;
    int64_t runs_per_row = kServeRunsPerRow;
    int64_t slab_planes = kSlabPlanes, store_permille = kStorePermille;
    size_t bytes_of(const Geom& g, roix_dtype dt, roix_eb eb, const roix_criterion* crit) const {
        if (compact_of(dt, eb, crit)) return compact_plan(g, slab_planes, store_permille, runs_per_row).total;
        return volume_bytes(g, dt, incremental_of(eb, crit), runs_per_row, ctx->p16_min);
    }
    int64_t admitted = 0, refused = 0, slabs_done = 0, closes_done = 0, bytes_in = 0;
    std::vector<double> slab_lat, close_lat;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    hipEvent_t event() {
        if (!events.empty()) {
            hipEvent_t e = events.back();
            events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void release(Vol& v) {
        pool.release(v.off, v.bytes);
        v.bytes = 0;
        if (v.stage_free) {
            hipEventDestroy(v.stage_free);
            v.stage_free = nullptr;
        }
    }
    // Account for every request and aborted volume whose events completed.
    void reap() {
        for (auto& kv : reqs) {
            Req& r = kv.second;
            if (r.finished) continue;
            const hipError_t q = hipEventQuery(r.done);
            if (q == hipErrorNotReady) continue;
            r.finished = true;
            r.status = q == hipSuccess ? ROIX_OK : ROIX_EDEVICE;
            float ms = 0.0f;
            if (q == hipSuccess && hipEventElapsedTime(&ms, ev_ref, r.done) == hipSuccess)
                r.done_ms = (double)ms;
            else
                r.done_ms = now_ms();
            const double lat = r.done_ms - r.submit_ms;
            if (r.kind == ROIX_REQ_SLAB) {
                ++slabs_done;
                slab_lat.push_back(lat);
            } else {
                ++closes_done;
                close_lat.push_back(lat);
                auto it = vols.find(r.vol);
                if (it != vols.end()) {
                    release(it->second);
                    vols.erase(it);
                }
            }
        }
        for (auto it = vols.begin(); it != vols.end();) {
            Vol& v = it->second;
            if (v.state == V_ABORTED && hipEventQuery(v.release_ev) != hipErrorNotReady) {
                events.push_back(v.release_ev);
                release(v);
                it = vols.erase(it);
            } else {
                ++it;
            }
        }
    }
};

// --------------------------------------------------------- launch sequences

static hipError_t enqueue_slab(const LaunchCtx& lc, Vol& v, int64_t z0, int64_t nzs) {
    const Geom& g = v.g;
    const Layout& L = v.L;
    const int64_t r0 = z0 * g.ny, r1 = (z0 + nzs) * g.ny;
    hipError_t e;
    if ((e = launch_slab_mask(lc, v.d_vol, v.dt, g, r0, r1, L)) != hipSuccess) return e;
    if ((e = launch_scan_u32_base(lc, L.row_nruns + r0, L.run_off + r0, r1 - r0, &L.S->n_runs, &L.S->seg_lo,
                                  L.run_off + r1, L.scan_tmp, L.S, L.run_cap, ROIX_ENOMEM)) != hipSuccess)
        return e;
    if ((e = launch_runs_write(lc, g, L, r0, r1)) != hipSuccess) return e;
    return launch_union(lc, g, L, v.crit.connectivity);
}

// A staged chunk of planes [z0, z0 + nzs) of a volume kept as row extents:
// the slab kernels on the stage (the input and bitmask pointers shifted so
// that absolute row numbers land in the stage), then the code classes and
// the store of the rows' extents.
static hipError_t enqueue_slab_compact(const LaunchCtx& lc, Vol& v, int64_t z0, int64_t nzs) {
    const Geom& g = v.g;
    const int64_t r0 = z0 * g.ny, r1 = (z0 + nzs) * g.ny;
    Layout L = v.L;
    L.maskbits = (uint64_t*)((uintptr_t)v.L.maskbits - (uintptr_t)(r0 * g.W * 8));
    const uint16_t* in = (const uint16_t*)((uintptr_t)v.stage - (uintptr_t)(r0 * g.nx * 2));
    hipError_t e;
    if ((e = launch_slab_mask(lc, in, ROIX_U16, g, r0, r1, L)) != hipSuccess) return e;
    if ((e = launch_scan_u32_base(lc, L.row_nruns + r0, L.run_off + r0, r1 - r0, &L.S->n_runs, &L.S->seg_lo,
                                  L.run_off + r1, L.scan_tmp, L.S, L.run_cap, ROIX_ENOMEM)) != hipSuccess)
        return e;
    if ((e = launch_runs_write(lc, g, L, r0, r1)) != hipSuccess) return e;
    if ((e = launch_union(lc, g, L, v.crit.connectivity)) != hipSuccess) return e;
    if ((e = launch_slab_classes(lc, v.stage, (uint64_t)nzs * (uint64_t)g.ny * (uint64_t)g.nx, L.S, v.classes)) !=
        hipSuccess)
        return e;
    return launch_store_rows(lc, g, L, v.stage, r0, r1, v.store, v.store_cap, v.row_org, v.lens);
}

// The close of a volume kept as row extents: the quantiser and the histogram
// from the slabs' range and class counts, then the rest of the path reading
// the span values from the store.
static roix_status enqueue_close_compact(const LaunchCtx& lc, Vol& v) {
    DevState* S = v.L.S;
    ROIX_TRY(launch_serve_status(lc, S, 1));
    ROIX_TRY(launch_serve_resolve(lc, S, v.eb.value, v.crit.fixed_value, v.classes));
    ROIX_TRY(launch_otsu(lc, S, true));
    ROIX_TRY(launch_serve_status(lc, S, 0));
    ROIX_TRY(components_and_keep(lc, v.g, v.L, &v.crit, v.out.d_comps, v.out.comps_cap));
    ROIX_TRY(launch_spans_from_runs(lc, v.g, v.L));
    ROIX_TRY(spans_and_emit(lc, v.g, v.L, v.store, ROIX_U16, &v.out));
    ROIX_TRY(launch_finalize(lc, S, v.out.d_qinfo, v.out.d_sinfo, v.out.d_einfo, true));
    return ROIX_OK;
}

// The stages of the fused path that need the whole volume.  The quantiser
// stages (resolve, histogram, threshold) run with any run-capacity error of
// the slabs held back, so that errors are reported in the fused path's order.
static roix_status enqueue_close_incremental(const LaunchCtx& lc, Vol& v) {
    DevState* S = v.L.S;
    ROIX_TRY(launch_serve_status(lc, S, 1));
    ROIX_TRY(launch_resolve_dt(lc, S, v.dt, v.eb, &v.crit));
    ROIX_TRY(launch_hist_only(lc, v.d_vol, v.dt, v.g, S));
    ROIX_TRY(launch_otsu(lc, S, true));
    ROIX_TRY(launch_serve_status(lc, S, 0));
    ROIX_TRY(components_and_keep(lc, v.g, v.L, &v.crit, v.out.d_comps, v.out.comps_cap));
    ROIX_TRY(launch_spans_from_runs(lc, v.g, v.L));
    ROIX_TRY(spans_and_emit(lc, v.g, v.L, v.d_vol, v.dt, &v.out));
    ROIX_TRY(launch_finalize(lc, S, v.out.d_qinfo, v.out.d_sinfo, v.out.d_einfo, true));
    return ROIX_OK;
}

static LaunchCtx serve_lctx(roix_server* s) {
    LaunchCtx lc = lctx(s->ctx, s->compute);
    lc.timer = nullptr;
    return lc;
}

// ---------------------------------------------------------------------- ABI

extern "C" {

size_t roix_server_volume_bytes(const roix_server* s, roix_dims dims, roix_dtype dtype, roix_eb eb,
                                const roix_criterion* crit) {
    Geom g;
    if (!s || (dtype != ROIX_F32 && dtype != ROIX_U16) || !geom_of(dims, &g) || !eb_ok(eb) || !crit_ok(crit) ||
        crit->thr == ROIX_THR_OTSU_SLICE)
        return 0;
    return s->bytes_of(g, dtype, eb, crit);
}

roix_status roix_server_set_param(roix_server* s, const char* name, int64_t value) {
    if (!s || !name) return ROIX_EINVAL;
    if (strcmp(name, "runs_per_row") == 0 && value >= 1 && value <= (1ll << 30)) {
        s->runs_per_row = value;
        return ROIX_OK;
    }
    if (strcmp(name, "slab_planes") == 0 && value >= 1 && value <= 4096) {
        s->slab_planes = value;
        return ROIX_OK;
    }
    if (strcmp(name, "store_permille") == 0 && value >= 1 && value <= 1000) {
        s->store_permille = value;
        return ROIX_OK;
    }
    return ROIX_EINVAL;
}

roix_status roix_server_create(roix_ctx* ctx, size_t hbm_budget_bytes, roix_server** out) {
    if (!ctx || !out || hbm_budget_bytes < 256) return ROIX_EINVAL;
    *out = nullptr;
    DeviceGuard dg(ctx->device);
    roix_server* s = new (std::nothrow) roix_server();
    if (!s) return ROIX_ENOMEM;
    s->ctx = ctx;
    s->pool.init(hbm_budget_bytes);
    if (hipMalloc(&s->base, s->pool.size) != hipSuccess) {
        delete s;
        return ROIX_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev_ref) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_copy, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(s->ev_ref, s->compute) != hipSuccess || hipEventSynchronize(s->ev_ref) != hipSuccess) {
        roix_server_destroy(s);
        return ROIX_EDEVICE;
    }
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return ROIX_OK;
}

roix_status roix_server_destroy(roix_server* s) {
    if (!s) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    if (s->copy) hipStreamSynchronize(s->copy);
    if (s->compute) hipStreamSynchronize(s->compute);
    for (auto& kv : s->reqs)
        if (kv.second.done) hipEventDestroy(kv.second.done);
    for (auto& kv : s->vols) {
        if (kv.second.release_ev) hipEventDestroy(kv.second.release_ev);
        if (kv.second.stage_free) hipEventDestroy(kv.second.stage_free);
    }
    for (hipEvent_t e : s->events) hipEventDestroy(e);
    if (s->ev_ref) hipEventDestroy(s->ev_ref);
    if (s->ev_copy) hipEventDestroy(s->ev_copy);
    if (s->copy) hipStreamDestroy(s->copy);
    if (s->compute) hipStreamDestroy(s->compute);
    if (s->base) hipFree(s->base);
    delete s;
    return ROIX_OK;
}

roix_status roix_volume_open(roix_server* s, roix_dims dims, roix_dtype dtype, roix_eb eb,
                             const roix_criterion* crit, const roix_fused_out* final_out, int64_t* vol_id) {
    if (!s || !vol_id || !eb_ok(eb) || !crit_ok(crit) || !out_ok(final_out, true)) return ROIX_EINVAL;
    if (crit->thr == ROIX_THR_OTSU_SLICE) return ROIX_EINVAL;  // slabs are thresholded as they arrive
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    Geom g;
    if (!geom_of(dims, &g)) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    s->reap();
    Vol v;
    v.g = g;
    v.dt = dtype;
    v.eb = eb;
    v.crit = *crit;
    v.out = *final_out;
    v.incremental = incremental_of(eb, crit);
    v.compact = compact_of(dtype, eb, crit);
    v.bytes = s->bytes_of(g, dtype, eb, crit);
    if (!s->pool.alloc(v.bytes, &v.off)) {
        ++s->refused;
        return ROIX_EBUSY;
    }
    uint8_t* region = (uint8_t*)s->base + v.off;
    if (v.compact) {
        const CompactPlan p = compact_plan(g, s->slab_planes, s->store_permille, s->runs_per_row);
        v.stage_planes = s->slab_planes < g.nz ? s->slab_planes : g.nz;
        v.stage = (uint16_t*)(region + p.stage);
        v.store = (uint16_t*)(region + p.store);
        v.store_cap = p.store_cap;
        v.row_org = (uint64_t*)(region + p.row_org);
        v.lens = (uint64_t*)(region + p.lens);
        v.classes = (unsigned long long*)(region + p.classes);
        if (!carve_at(region + p.layout, p.total - p.layout, g, &v.L, 0, v.stage_planes * g.ny)) {
            s->release(v);
            return ROIX_ENOMEM;
        }
        v.L.row_org = v.row_org;
        v.L.nvals = v.store_cap;
        if (hipEventCreateWithFlags(&v.stage_free, hipEventDisableTiming) != hipSuccess) {
            v.stage_free = nullptr;
            s->release(v);
            return ROIX_EDEVICE;
        }
    } else {
        v.d_vol = region;
        const size_t in_bytes = align256((size_t)g.N * (dtype == ROIX_F32 ? 4 : 2));
        if (!carve_at(v.d_vol + in_bytes, v.bytes - in_bytes, g, &v.L,
                      v.incremental ? 0 : proxy_kind(g, dtype, s->ctx->p16_min))) {
            s->release(v);
            return ROIX_ENOMEM;
        }
    }
    const LaunchCtx lc = serve_lctx(s);
    if (launch_init(lc, v.L.S) != hipSuccess ||
        (v.incremental && launch_serve_open(lc, v.L.S, eb.value, crit->fixed_value) != hipSuccess) ||
        (v.compact && launch_store_open(lc, v.L.S, v.classes) != hipSuccess)) {
        s->release(v);
        return ROIX_EDEVICE;
    }
    const int64_t id = s->next_vol++;
    s->vols.emplace(id, v);
    ++s->admitted;
    *vol_id = id;
    return ROIX_OK;
}

roix_status roix_slab_submit(roix_server* s, int64_t vol_id, int64_t z0, int64_t nz_slab, const void* ptr,
                             int ptr_is_device, int64_t* req_id) {
    if (!s || !ptr || !req_id) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    s->reap();
    auto it = s->vols.find(vol_id);
    if (it == s->vols.end()) return ROIX_EINVAL;
    Vol& v = it->second;
    if (nz_slab < 1 || z0 < 0 || z0 + nz_slab > v.g.nz) return ROIX_EINVAL;
    if (v.state != V_OPEN || z0 != v.next_z) return ROIX_ESEQ;
    Req r;
    r.vol = vol_id;
    r.kind = ROIX_REQ_SLAB;
    r.submit_ms = s->now_ms();
    r.done = s->event();
    if (!r.done) return ROIX_EDEVICE;
    const size_t vb = v.dt == ROIX_F32 ? 4 : 2;
    const size_t plane = (size_t)v.g.nx * (size_t)v.g.ny * vb;
    const size_t bytes = plane * (size_t)nz_slab;
    const hipMemcpyKind kind = ptr_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipSuccess;
    if (v.compact) {
        // staged chunk by chunk: a copy into the stage waits until the
        // compute of the chunk before it has read the stage
        const LaunchCtx lc = serve_lctx(s);
        for (int64_t p = 0; p < nz_slab && e == hipSuccess; p += v.stage_planes) {
            const int64_t n = nz_slab - p < v.stage_planes ? nz_slab - p : v.stage_planes;
            e = hipStreamWaitEvent(s->copy, v.stage_free, 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(v.stage, (const uint8_t*)ptr + plane * (size_t)p, plane * (size_t)n, kind, s->copy);
            if (e == hipSuccess) e = hipEventRecord(s->ev_copy, s->copy);
            if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, s->ev_copy, 0);
            if (e == hipSuccess) e = enqueue_slab_compact(lc, v, z0 + p, n);
            if (e == hipSuccess) e = hipEventRecord(v.stage_free, s->compute);
        }
        if (e == hipSuccess) e = hipEventRecord(r.done, s->compute);
    } else {
        e = hipMemcpyAsync(v.d_vol + plane * (size_t)z0, ptr, bytes, kind, s->copy);
        if (v.incremental) {
            if (e == hipSuccess) e = hipEventRecord(s->ev_copy, s->copy);
            if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, s->ev_copy, 0);
            if (e == hipSuccess) e = enqueue_slab(serve_lctx(s), v, z0, nz_slab);
            if (e == hipSuccess) e = hipEventRecord(r.done, s->compute);
        } else if (e == hipSuccess) {
            e = hipEventRecord(r.done, s->copy);  // nothing to compute before the close
        }
    }
    if (e != hipSuccess) {
        s->events.push_back(r.done);
        return ROIX_EDEVICE;
    }
    v.next_z = z0 + nz_slab;
    s->bytes_in += (int64_t)bytes;
    const int64_t id = s->next_req++;
    s->reqs.emplace(id, r);
    *req_id = id;
    return ROIX_OK;
}

roix_status roix_volume_close(roix_server* s, int64_t vol_id, int64_t* req_id) {
    if (!s || !req_id) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    s->reap();
    auto it = s->vols.find(vol_id);
    if (it == s->vols.end()) return ROIX_EINVAL;
    Vol& v = it->second;
    if (v.state != V_OPEN || v.next_z != v.g.nz) return ROIX_ESEQ;
    Req r;
    r.vol = vol_id;
    r.kind = ROIX_REQ_CLOSE;
    r.submit_ms = s->now_ms();
    r.done = s->event();
    if (!r.done) return ROIX_EDEVICE;
    const LaunchCtx lc = serve_lctx(s);
    roix_status st = ROIX_OK;
    // the copy stream is in order: waiting for its latest point covers every slab
    if (hipEventRecord(s->ev_copy, s->copy) != hipSuccess || hipStreamWaitEvent(s->compute, s->ev_copy, 0) != hipSuccess)
        st = ROIX_EDEVICE;
    if (st == ROIX_OK)
        st = v.compact       ? enqueue_close_compact(lc, v)
             : v.incremental ? enqueue_close_incremental(lc, v)
                             : enqueue_fused(lc, v.g, v.L, v.d_vol, v.dt, v.eb, &v.crit, &v.out);
    if (st == ROIX_OK && hipEventRecord(r.done, s->compute) != hipSuccess) st = ROIX_EDEVICE;
    if (st != ROIX_OK) {
        s->events.push_back(r.done);
        return st;
    }
    v.state = V_CLOSING;
    const int64_t id = s->next_req++;
    s->reqs.emplace(id, r);
    *req_id = id;
    return ROIX_OK;
}

roix_status roix_volume_abort(roix_server* s, int64_t vol_id) {
    if (!s) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    s->reap();
    auto it = s->vols.find(vol_id);
    if (it == s->vols.end()) return ROIX_EINVAL;
    Vol& v = it->second;
    if (v.state != V_OPEN) return ROIX_ESEQ;
    // released once every copy and kernel enqueued so far has finished
    hipEvent_t ev = s->event();
    if (!ev || hipEventRecord(s->ev_copy, s->copy) != hipSuccess ||
        hipStreamWaitEvent(s->compute, s->ev_copy, 0) != hipSuccess || hipEventRecord(ev, s->compute) != hipSuccess) {
        if (ev) s->events.push_back(ev);
        return ROIX_EDEVICE;
    }
    v.release_ev = ev;
    v.state = V_ABORTED;
    return ROIX_OK;
}

roix_status roix_wait(roix_server* s, int64_t req_id, int64_t timeout_ms, roix_req_result* res) {
    if (!s || !res) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return ROIX_EINVAL;
    const auto start = std::chrono::steady_clock::now();
    while (true) {
        s->reap();
        Req& r = it->second;
        if (r.finished) {
            res->status = r.status;
            res->kind = r.kind;
            res->vol_id = r.vol;
            res->submit_ms = r.submit_ms;
            res->done_ms = r.done_ms;
            res->latency_ms = r.done_ms - r.submit_ms;
            s->events.push_back(r.done);
            s->reqs.erase(it);
            return ROIX_OK;
        }
        if (timeout_ms >= 0 &&
            std::chrono::steady_clock::now() - start >= std::chrono::milliseconds(timeout_ms))
            return ROIX_EBUSY;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

roix_status roix_server_stats(roix_server* s, roix_server_stats_t* o) {
    if (!s || !o) return ROIX_EINVAL;
    DeviceGuard dg(s->ctx->device);
    s->reap();
    o->volumes_admitted = s->admitted;
    o->volumes_refused = s->refused;
    o->volumes_open = 0;
    for (auto& kv : s->vols)
        if (kv.second.state == V_OPEN) ++o->volumes_open;
    o->slabs_done = s->slabs_done;
    o->closes_done = s->closes_done;
    o->bytes_in = s->bytes_in;
    o->budget_bytes = s->pool.size;
    o->bytes_in_use = s->pool.used;
    o->slab_p50_ms = pct(s->slab_lat, 0.50);
    o->slab_p99_ms = pct(s->slab_lat, 0.99);
    o->slab_max_ms = s->slab_lat.empty() ? 0.0 : *std::max_element(s->slab_lat.begin(), s->slab_lat.end());
    o->close_p50_ms = pct(s->close_lat, 0.50);
    o->close_p99_ms = pct(s->close_lat, 0.99);
    return ROIX_OK;
}

}  // extern "C"
