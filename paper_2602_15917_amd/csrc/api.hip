// api.hip - the C ABI of libroix.so: context and scratch arena, argument
// checks, the launch sequences of the quantise / segment / extract / fused
// calls, and per-stage event timing.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "host.h"

namespace roix {

void timer_begin(Timer* t, int stage, hipStream_t s) {
    if (!t || !t->on) return;
    hipEvent_t e = t->get();
    if (!e) return;
    hipEventRecord(e, s);
    t->open[stage].a = e;
}

void timer_end(Timer* t, int stage, hipStream_t s) {
    if (!t || !t->on || !t->open[stage].a) return;
    hipEvent_t e = t->get();
    if (!e) return;
    hipEventRecord(e, s);
    t->pending.push_back({stage, t->open[stage].a, e});
    t->open[stage].a = nullptr;
}

static const char* kStageNames[ST_COUNT] = {
    "init", "range", "resolve", "quantize", "quant_hist", "quant_range16", "otsu", "mask_runs", "scan", "runs_write",
    "union", "flatten", "comp_stats", "keep", "spans", "emit", "emit_rows", "voxel_out", "finalize", "decode_index", "decode", "background", "abs_quantize", "huffman", "section"};

}  // namespace roix

using namespace roix;

// ----------------------------------------------------------------- layout

size_t roix::align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool roix::geom_of(roix_dims d, Geom* g) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return false;
    if (d.nx > (1ll << 31) - 64 || d.ny > (1ll << 31) || d.nz > (1ll << 31)) return false;
    const unsigned __int128 n = (unsigned __int128)d.nx * d.ny * d.nz;
    if (n > ((unsigned __int128)1 << 33)) return false;
    if ((unsigned __int128)d.ny * d.nz >= ((unsigned __int128)1 << 31)) return false;
    g->nx = d.nx;
    g->ny = d.ny;
    g->nz = d.nz;
    g->N = (uint64_t)n;
    g->nrows = d.ny * d.nz;
    g->W = (d.nx + 63) / 64;
    return true;
}


uint64_t roix::worst_runs(const Geom& g) {
    uint64_t w = (uint64_t)g.nrows * (uint64_t)((g.nx + 1) / 2);
    const uint64_t cap = (1ull << 31) - 1;
    return w < cap ? w : cap;
}

int roix::proxy_kind(const Geom& g, roix_dtype dt, uint64_t min_voxels) {
    return (dt == ROIX_F32 && g.N >= min_voxels && g.nx % 4 == 0) ? 2 : 1;
}

int roix::proxy_kind_for(const Geom& g, roix_dtype dt, size_t bytes, uint64_t min_voxels) {
    const int k = proxy_kind(g, dt, min_voxels);
    return (k == 2 && bytes < fixed_bytes(g, 2) + (size_t)worst_runs(g) * kRunBytes) ? 1 : k;
}

// bytes of the per-voxel and per-row part of the arena
size_t roix::fixed_bytes(const Geom& g, int proxy, int64_t mask_rows) {
    const int64_t mrows = mask_rows < 0 ? g.nrows : mask_rows;
    size_t b = 0;
    b += align256(sizeof(DevState));
    if (proxy) b += align256((size_t)g.nrows * g.W * 64 * (proxy == 2 ? 2 : 1));  // proxy
    if (proxy == 2) b += align256((size_t)kQrBlocks * kQrFine * 4) + align256((size_t)kQrFine * 8);
    b += align256((size_t)mrows * g.W * 8);               // mask bits
    b += align256((size_t)g.nrows * 4);                   // row_nruns
    b += align256((size_t)(g.nrows + 1) * 4);             // run_off
    b += 2 * align256((size_t)g.nrows * 4);               // row_xs, row_xe
    b += align256((size_t)g.nrows * 8);                   // row_packed
    b += align256((size_t)g.nrows * 8);                   // row_outl
    b += align256((size_t)g.nrows * 4);                   // nz_rows
    b += align256((size_t)g.nrows * 16);                  // span_desc
    b += 2 * align256((size_t)(g.N / kEmitChunk + 2) * 4);  // chunk_row, slow_chunks
    b += align256((size_t)(kScanBlocks + 1) * 8);         // scan tmp
    b += align256((size_t)g.nz * 4);                      // slice_thr
    b += 6 * 256;                                         // run-array alignment slack
    return b;
}

bool roix::carve_at(void* base, size_t bytes, const Geom& g, Layout* L, int proxy, int64_t mask_rows) {
    const size_t fb = fixed_bytes(g, proxy, mask_rows);
    const int64_t mrows = mask_rows < 0 ? g.nrows : mask_rows;
    if (bytes < fb + kRunBytes) return false;
    uint8_t* p = (uint8_t*)base;
    auto take = [&](size_t n) {
        uint8_t* q = p;
        p += align256(n);
        return q;
    };
    L->S = (DevState*)take(sizeof(DevState));
    L->proxy = proxy ? take((size_t)g.nrows * g.W * 64 * (proxy == 2 ? 2 : 1)) : nullptr;
    L->fine_slots = proxy == 2 ? (uint32_t*)take((size_t)kQrBlocks * kQrFine * 4) : nullptr;
    L->fine_total = proxy == 2 ? (unsigned long long*)take((size_t)kQrFine * 8) : nullptr;
    L->maskbits = (uint64_t*)take((size_t)mrows * g.W * 8);
    L->row_nruns = (uint32_t*)take((size_t)g.nrows * 4);
    L->run_off = (uint32_t*)take((size_t)(g.nrows + 1) * 4);
    L->row_xs = (uint32_t*)take((size_t)g.nrows * 4);
    L->row_xe = (uint32_t*)take((size_t)g.nrows * 4);
    L->row_packed = (uint64_t*)take((size_t)g.nrows * 8);
    L->row_outl = (uint64_t*)take((size_t)g.nrows * 8);
    L->nz_rows = (uint32_t*)take((size_t)g.nrows * 4);
    L->span_desc = (uint64_t*)take((size_t)g.nrows * 16);
    L->chunk_row = (uint32_t*)take((size_t)(g.N / kEmitChunk + 2) * 4);
    L->slow_chunks = (uint32_t*)take((size_t)(g.N / kEmitChunk + 2) * 4);
    L->scan_tmp = (uint64_t*)take((size_t)(kScanBlocks + 1) * 8);
    L->slice_thr = (int32_t*)take((size_t)g.nz * 4);
    const size_t used = (size_t)(p - (uint8_t*)base) + 6 * 256;
    uint64_t cap = (bytes - used) / kRunBytes;
    const uint64_t w = worst_runs(g);
    if (cap > w) cap = w;
    if (cap < 1) return false;
    L->run_cap = cap;
    L->row_org = nullptr;
    L->nvals = 0;
    L->run_xs = (uint32_t*)take(cap * 4);
    L->run_xe = (uint32_t*)take(cap * 4);
    L->parent = (uint32_t*)take(cap * 4);
    L->comp_id = (uint32_t*)take(cap * 4);
    L->run_row = (uint32_t*)take(cap * 4);
    L->kept_flag = (uint8_t*)take(cap);
    return (size_t)(p - (uint8_t*)base) <= bytes;
}

static bool carve(roix_ctx* c, const Geom& g, Layout* L, roix_dtype dt = ROIX_U16) {
    return carve_at(c->arena, c->arena_bytes, g, L, proxy_kind_for(g, dt, c->arena_bytes, c->p16_min));
}

LaunchCtx roix::lctx(roix_ctx* c, void* stream) {
    LaunchCtx lc;
    lc.stream = (hipStream_t)stream;
    lc.timer = c->timer.on ? &c->timer : nullptr;
    lc.grid_stream = c->grid_stream;
    lc.grid_read = c->grid_read;
    lc.grid_emit = c->grid_emit;
    lc.grid_mask = c->grid_mask;
    lc.seg_grid = c->seg_grid;
    lc.seg_runs = c->seg_runs;
    lc.stats_grid = c->stats_grid;
    lc.cus = c->cus;
    return lc;
}

bool roix::aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool roix::eb_ok(roix_eb eb) {
    return (eb.mode == ROIX_EB_ABS || eb.mode == ROIX_EB_REL) && eb.value > 0.0 && eb.value <= 1.7976931348623157e308;
}

bool roix::crit_ok(const roix_criterion* c) {
    if (!c) return false;
    if (c->thr != ROIX_THR_OTSU && c->thr != ROIX_THR_FIXED && c->thr != ROIX_THR_MULTI_OTSU &&
        c->thr != ROIX_THR_OTSU_SLICE)
        return false;
    if (c->thr == ROIX_THR_MULTI_OTSU && c->classes != 0 && c->classes != 3 && c->classes != 4) return false;
    if (c->thr == ROIX_THR_FIXED && !(c->fixed_value >= -1.7976931348623157e308 && c->fixed_value <= 1.7976931348623157e308))
        return false;
    if (c->connectivity != 6 && c->connectivity != 26) return false;
    if (c->keep != ROIX_KEEP_MIN_SIZE && c->keep != ROIX_KEEP_LARGEST) return false;
    if (c->keep == ROIX_KEEP_MIN_SIZE && c->min_size < 1) return false;
    return true;
}

bool roix::out_ok(const roix_fused_out* o, bool need_comps) {
    if (!o) return false;
    if (o->rows_cap < 0 || o->stream_cap_bytes < 0 || o->outliers_cap < 0 || o->comps_cap < 0) return false;
    if (o->rows_cap > 0 && (!o->d_rows || !aligned(o->d_rows, 8))) return false;
    if (o->stream_cap_bytes > 0 && (!o->d_stream || !aligned(o->d_stream, 4))) return false;
    if (o->outliers_cap > 0 && (!o->d_outliers || !aligned(o->d_outliers, 4))) return false;
    if (need_comps && o->comps_cap > 0 && (!o->d_comps || !aligned(o->d_comps, 8))) return false;
    return true;
}

static roix_status dev_err(hipError_t e) { return e == hipSuccess ? ROIX_OK : ROIX_EDEVICE; }


// --------------------------------------------------------- shared stages

// mask -> runs -> union of a whole volume (everything between the proxy and
// the flattening)
static hipError_t label_runs(const LaunchCtx& lc, const Geom& g, const Layout& L, int connectivity,
                             const int32_t* slice_thr = nullptr, const uint16_t* u16_in = nullptr) {
    hipError_t e;
    if ((e = launch_mask_runs(lc, g, L, slice_thr, u16_in)) != hipSuccess) return e;
    if ((e = launch_scan_u32(lc, L.row_nruns, L.run_off, g.nrows, nullptr, &L.S->n_runs, L.run_off + g.nrows,
                             L.scan_tmp, L.S, L.run_cap, ROIX_ENOMEM)) != hipSuccess)
        return e;
    if ((e = launch_runs_write(lc, g, L, 0, g.nrows)) != hipSuccess) return e;
    return launch_union(lc, g, L, connectivity);
}

// flatten -> component ids and entries -> stats -> keep
hipError_t roix::components_and_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, const roix_criterion* crit,
                                     roix_component* comps, int64_t comps_cap) {
    hipError_t e;
    if ((e = launch_flatten(lc, g, L)) != hipSuccess) return e;
    const uint64_t cap = (uint64_t)(comps ? comps_cap : 0);
    const CompInit ci{L.run_xs, L.run_row, g.nx, comps, L.kept_flag, cap};
    if ((e = launch_scan_u32(lc, L.comp_id, L.comp_id, (int64_t)L.run_cap, &L.S->n_runs, &L.S->n_comps, nullptr,
                             L.scan_tmp, L.S, cap, ROIX_ETRUNC, &ci)) != hipSuccess)
        return e;
    if ((e = launch_comp_stats(lc, g, L, comps)) != hipSuccess) return e;
    return launch_keep(lc, g, L, comps, crit);
}

static hipError_t label_and_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, const roix_criterion* crit,
                                 roix_component* comps, int64_t comps_cap, const uint16_t* u16_in = nullptr) {
    hipError_t e;
    const int32_t* st = crit->thr == ROIX_THR_OTSU_SLICE ? L.slice_thr : nullptr;
    if ((e = label_runs(lc, g, L, crit->connectivity, st, u16_in)) != hipSuccess) return e;
    return components_and_keep(lc, g, L, crit, comps, comps_cap);
}

hipError_t roix::spans_and_emit(const LaunchCtx& lc, const Geom& g, const Layout& L, const void* in, roix_dtype dt,
                                 const roix_fused_out* out, const BgRef* bg) {
    hipError_t e;
    if ((e = launch_scan_u64(lc, L.row_packed, L.row_packed, g.nrows, &L.S->span_total, L.scan_tmp)) != hipSuccess)
        return e;
    return launch_emit(lc, g, L, in, dt, out, bg);
}

// the launch sequence of the fused path on an already carved layout
roix_status roix::enqueue_fused(const LaunchCtx& lc, const Geom& g, Layout L, const void* d_in, roix_dtype dtype,
                                 roix_eb eb, const roix_criterion* crit, const roix_fused_out* out) {
    const bool fixed = crit->thr == ROIX_THR_FIXED;
    const int kind = dtype == ROIX_F32 ? 0 : 1;
    // the fused range + 16-bit proxy pass needs the bound before the range
    // (absolute) and whole 16-byte vectors per row
    // per-slice thresholds compare 1-byte bins slice by slice: the two-pass flow
    const bool per_slice = crit->thr == ROIX_THR_OTSU_SLICE;
    const bool p16 = !per_slice && L.fine_slots && dtype == ROIX_F32 && eb.mode == ROIX_EB_ABS && aligned(d_in, 16);
    // a uint16 volume of whole 64-voxel rows needs no proxy: the histogram
    // pass only counts, and the mask pass compares the values themselves
    // with the smallest value whose code reaches the threshold
    const bool u16_direct = !per_slice && dtype == ROIX_U16 && g.W * 64 == g.nx && aligned(d_in, 16);
    if (p16) {
        ROIX_TRY(launch_init(lc, L.S, eb.value));
        ROIX_TRY(launch_quant_range16(lc, (const float*)d_in, g, L));
        ROIX_TRY(launch_resolve16(lc, L, eb, crit));
        ROIX_TRY(launch_quant_hist(lc, d_in, kind, g, L.S, L.proxy, fixed, true));  // only when K > 2^15
    } else {
        ROIX_TRY(launch_init(lc, L.S));
        ROIX_TRY(launch_range(lc, d_in, dtype, g.N, L.S));
        ROIX_TRY(launch_resolve_dt(lc, L.S, dtype, eb, crit));
        if (u16_direct)
            ROIX_TRY(launch_hist_only(lc, d_in, dtype, g, L.S));
        else
            ROIX_TRY(launch_quant_hist(lc, d_in, kind, g, L.S, L.proxy, fixed));
    }
    if (per_slice)
        ROIX_TRY(launch_slice_otsu(lc, g, L.proxy, L.S, L.slice_thr, out->d_slice_thr));
    else
        ROIX_TRY(launch_threshold(lc, L.S, crit));
    ROIX_TRY(label_and_keep(lc, g, L, crit, out->d_comps, out->comps_cap,
                            u16_direct ? (const uint16_t*)d_in : nullptr));
    ROIX_TRY(launch_spans_from_runs(lc, g, L));
    ROIX_TRY(spans_and_emit(lc, g, L, d_in, dtype, out));
    ROIX_TRY(launch_finalize(lc, L.S, out->d_qinfo, out->d_sinfo, out->d_einfo, true));
    return ROIX_OK;
}

// The fused path on M = I - B.  With the one-pass flow and the 16-bit proxy
// (rows of whole 64-voxel words) the range/code pass reads I and B and the
// row-table kernel gathers outlier values as I - B: M is never written.  M
// goes to bg.work only where a stage must read it: when the range pass falls
// back to the 1-byte proxy (K > 2^15), or when the proxy emit queued chunks
// for the general kernel.  Any other case subtracts first and runs the path
// on bg.work.
roix_status roix::enqueue_fused_bg(const LaunchCtx& lc, const Geom& g, Layout L, const float* d_in, const BgRef& bg,
                                    roix_eb eb, const roix_criterion* crit, const roix_fused_out* out) {
    const bool fused = crit->thr != ROIX_THR_OTSU_SLICE && L.fine_slots && eb.mode == ROIX_EB_ABS &&
                       aligned(d_in, 16) && aligned(bg.bg, 16) && g.W * 64 == g.nx;
    if (!fused) {
        ROIX_TRY(launch_background(lc, d_in, ROIX_F32, bg.bg, !bg.plane, g, ROIX_BG_SUBTRACT, bg.work));
        return enqueue_fused(lc, g, L, bg.work, ROIX_F32, eb, crit, out);
    }
    const bool fixed = crit->thr == ROIX_THR_FIXED;
    ROIX_TRY(launch_init(lc, L.S, eb.value));
    ROIX_TRY(launch_quant_range16(lc, d_in, g, L, &bg));
    ROIX_TRY(launch_resolve16(lc, L, eb, crit));
    ROIX_TRY(launch_background_if(lc, d_in, bg, g, L.S, 1));
    ROIX_TRY(launch_quant_hist(lc, bg.work, 0, g, L.S, L.proxy, fixed, true));  // only when K > 2^15
    ROIX_TRY(launch_threshold(lc, L.S, crit));
    ROIX_TRY(label_and_keep(lc, g, L, crit, out->d_comps, out->comps_cap));
    ROIX_TRY(launch_spans_from_runs(lc, g, L));
    ROIX_TRY(spans_and_emit(lc, g, L, d_in, ROIX_F32, out, &bg));
    ROIX_TRY(launch_finalize(lc, L.S, out->d_qinfo, out->d_sinfo, out->d_einfo, true));
    return ROIX_OK;
}

// ------------------------------------------------------------------- ABI

extern "C" {

const char* roix_status_string(roix_status st) {
    switch (st) {
        case ROIX_OK: return "ok";
        case ROIX_EINVAL: return "invalid argument or input";
        case ROIX_ERANGE: return "codes out of exact fp32 range";
        case ROIX_ENOMEM: return "out of memory (scratch arena)";
        case ROIX_ETRUNC: return "output buffer too small";
        case ROIX_EDEVICE: return "device error";
        case ROIX_EBUSY: return "busy";
        case ROIX_ESEQ: return "out-of-sequence request";
    }
    return "unknown status";
}

size_t roix_sizeof(const char* t) {
    if (!t) return 0;
    struct {
        const char* n;
        size_t s;
    } const tab[] = {{"roix_quant_info", sizeof(roix_quant_info)},   {"roix_seg_info", sizeof(roix_seg_info)},
                     {"roix_extract_info", sizeof(roix_extract_info)}, {"roix_component", sizeof(roix_component)},
                     {"roix_row", sizeof(roix_row)},                   {"roix_fused_out", sizeof(roix_fused_out)},
                     {"roix_criterion", sizeof(roix_criterion)},       {"roix_eb", sizeof(roix_eb)},
                     {"roix_dims", sizeof(roix_dims)},                 {"roix_volume_desc", sizeof(roix_volume_desc)},
                     {"roix_req_result", sizeof(roix_req_result)},     {"roix_server_stats_t", sizeof(roix_server_stats_t)},
                     {"roix_decode_info", sizeof(roix_decode_info)},   {"roix_absq_info", sizeof(roix_absq_info)},
                     {"roix_huff_info", sizeof(roix_huff_info)},       {"roix_tune_result", sizeof(roix_tune_result)}};
    for (const auto& e : tab)
        if (strcmp(e.n, t) == 0) return e.s;
    return 0;
}

int roix_stage_count(void) { return ST_COUNT; }

const char* roix_stage_name(int stage) { return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : nullptr; }

size_t roix_scratch_bytes(roix_dims dims, roix_dtype dtype, const roix_criterion* crit) {
    (void)crit;
    Geom g;
    if ((dtype != ROIX_F32 && dtype != ROIX_U16) || !geom_of(dims, &g)) return 0;
    return fixed_bytes(g, proxy_kind(g, dtype)) + (size_t)worst_runs(g) * kRunBytes;
}

roix_status roix_bounds(roix_dims dims, roix_dtype dtype, const roix_criterion* crit, int64_t* max_rows,
                        int64_t* max_stream_bytes, int64_t* max_outliers, int64_t* max_components) {
    Geom g;
    if ((dtype != ROIX_F32 && dtype != ROIX_U16) || !geom_of(dims, &g)) return ROIX_EINVAL;
    if (max_rows) *max_rows = g.nrows;
    if (max_stream_bytes) *max_stream_bytes = (int64_t)(g.N * 4);
    if (max_outliers) *max_outliers = (int64_t)g.N;
    if (max_components) {
        const bool c26 = crit && crit->connectivity == 26;
        *max_components = c26 ? ((g.nx + 1) / 2) * ((g.ny + 1) / 2) * ((g.nz + 1) / 2) : (int64_t)g.N;
    }
    return ROIX_OK;
}

roix_status roix_ctx_create(int device, size_t scratch_bytes, roix_ctx** out) {
    if (!out) return ROIX_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ROIX_EINVAL;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return ROIX_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return ROIX_EDEVICE;
    roix_ctx* c = new (std::nothrow) roix_ctx();
    if (!c) return ROIX_ENOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cus = prop.multiProcessorCount;
    if (c->cus <= 0) c->cus = 256;
    c->grid_stream = c->cus * 8;
    c->grid_read = c->cus * 4;
    // the emit kernels run best with every wave resident at once (no
    // second, ragged round: the 16-bit-proxy emit kernel holds 6 waves per
    // SIMD, 6 workgroups of 4 waves per CU); the mask-word kernels with many
    // more
    c->grid_emit = c->cus * 6;
    c->grid_mask = c->cus * 32;
    c->seg_grid = c->cus * 2;
    c->stats_grid = c->cus;
    if (const char* s = getenv("ROIX_GRID_STREAM")) {
        int v = atoi(s);
        if (v > 0 && v <= 1 << 20) c->grid_stream = v;
    }
    if (const char* s = getenv("ROIX_GRID_READ")) {
        int v = atoi(s);
        if (v > 0 && v <= 1 << 20) c->grid_read = v;
    }
    c->arena_bytes = scratch_bytes ? scratch_bytes : ((size_t)1 << 30);
    if (hipMalloc(&c->arena, c->arena_bytes) != hipSuccess) {
        hipSetDevice(prev);
        delete c;
        return ROIX_ENOMEM;
    }
    hipSetDevice(prev);
    *out = c;
    return ROIX_OK;
}

roix_status roix_ctx_destroy(roix_ctx* ctx) {
    if (!ctx) return ROIX_EINVAL;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto& p : ctx->timer.pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    for (auto e : ctx->timer.pool) hipEventDestroy(e);
    batch_destroy(ctx->batch);
    hipFree(ctx->arena);
    hipSetDevice(prev);
    delete ctx;
    return ROIX_OK;
}

roix_status roix_ctx_set_timing(roix_ctx* ctx, int enable) {
    if (!ctx) return ROIX_EINVAL;
    ctx->timer.on = enable != 0;
    return ROIX_OK;
}

roix_status roix_ctx_read_timing(roix_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx) return ROIX_EINVAL;
    if (ms)
        for (int i = 0; i < ST_COUNT; ++i) ms[i] = 0.0;
    if (launches)
        for (int i = 0; i < ST_COUNT; ++i) launches[i] = 0;
    roix_status st = ROIX_OK;
    for (auto& p : ctx->timer.pending) {
        float t = 0.0f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&t, p.a, p.b) != hipSuccess)
            st = ROIX_EDEVICE;
        if (ms) ms[p.stage] += (double)t;
        if (launches) launches[p.stage] += 1;
        ctx->timer.pool.push_back(p.a);
        ctx->timer.pool.push_back(p.b);
    }
    ctx->timer.pending.clear();
    return st;
}

roix_status roix_quantize(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                          int32_t* d_codes, uint32_t* d_outlier_bits, roix_quant_info* d_qinfo, void* stream) {
    Geom g;
    if (!ctx || !d_in || !d_codes || !d_qinfo || !geom_of(dims, &g) || !eb_ok(eb)) return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (!aligned(d_in, dtype == ROIX_F32 ? 4 : 2) || !aligned(d_codes, 4) ||
        (d_outlier_bits && !aligned(d_outlier_bits, 4)))
        return ROIX_EINVAL;
    Layout L;
    if (!carve(ctx, g, &L)) return ROIX_ENOMEM;
    LaunchCtx lc = lctx(ctx, stream);
    ROIX_TRY(launch_init(lc, L.S));
    ROIX_TRY(launch_range(lc, d_in, dtype, g.N, L.S));
    ROIX_TRY(launch_resolve_dt(lc, L.S, dtype, eb, nullptr));
    ROIX_TRY(launch_quantize(lc, d_in, dtype, g.N, L.S, d_codes, d_outlier_bits));
    ROIX_TRY(launch_finalize(lc, L.S, d_qinfo, nullptr, nullptr, false));
    return ROIX_OK;
}

roix_status roix_segment(roix_ctx* ctx, const int32_t* d_codes, roix_dims dims, const roix_quant_info* d_qinfo,
                         const roix_criterion* crit, uint8_t* d_keep, int64_t* d_labels, roix_component* d_comps,
                         int64_t comps_cap, roix_seg_info* d_sinfo, void* stream) {
    Geom g;
    if (!ctx || !d_codes || !d_qinfo || !d_keep || !d_sinfo || !geom_of(dims, &g) || !crit_ok(crit) ||
        crit->thr == ROIX_THR_OTSU_SLICE)
        return ROIX_EINVAL;
    if (comps_cap < 0 || (comps_cap > 0 && (!d_comps || !aligned(d_comps, 8))) || !aligned(d_codes, 4) ||
        (d_labels && !aligned(d_labels, 8)))
        return ROIX_EINVAL;
    Layout L;
    if (!carve(ctx, g, &L)) return ROIX_ENOMEM;
    LaunchCtx lc = lctx(ctx, stream);
    const bool fixed = crit->thr == ROIX_THR_FIXED;
    ROIX_TRY(launch_init(lc, L.S));
    ROIX_TRY(launch_seg_init(lc, L.S, d_qinfo, crit));
    ROIX_TRY(launch_quant_hist(lc, d_codes, 2, g, L.S, L.proxy, fixed));
    ROIX_TRY(launch_threshold(lc, L.S, crit));
    ROIX_TRY(label_and_keep(lc, g, L, crit, d_comps, comps_cap));
    ROIX_TRY(launch_voxel_out(lc, g, L, d_comps, d_keep, d_labels));
    ROIX_TRY(launch_finalize(lc, L.S, nullptr, d_sinfo, nullptr, false));
    return ROIX_OK;
}

roix_status roix_extract(roix_ctx* ctx, const void* d_in, roix_dtype dtype, const uint8_t* d_keep, roix_dims dims,
                         const roix_quant_info* d_qinfo, const roix_fused_out* out, void* stream) {
    Geom g;
    if (!ctx || !d_in || !d_keep || !d_qinfo || !geom_of(dims, &g) || !out_ok(out, false)) return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (!aligned(d_in, dtype == ROIX_F32 ? 4 : 2)) return ROIX_EINVAL;
    Layout L;
    if (!carve(ctx, g, &L)) return ROIX_ENOMEM;
    LaunchCtx lc = lctx(ctx, stream);
    roix_criterion none;
    memset(&none, 0, sizeof none);
    none.thr = ROIX_THR_OTSU;
    ROIX_TRY(launch_init(lc, L.S));
    ROIX_TRY(launch_seg_init(lc, L.S, d_qinfo, &none));
    ROIX_TRY(launch_spans_from_keep(lc, g, L, d_keep));
    ROIX_TRY(spans_and_emit(lc, g, L, d_in, dtype, out));
    ROIX_TRY(launch_finalize(lc, L.S, nullptr, nullptr, out->d_einfo, false));
    return ROIX_OK;
}

roix_status roix_fused(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                       const roix_criterion* crit, const roix_fused_out* out, void* stream) {
    Geom g;
    if (!ctx || !d_in || !geom_of(dims, &g) || !eb_ok(eb) || !crit_ok(crit) || !out_ok(out, true))
        return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (!aligned(d_in, dtype == ROIX_F32 ? 4 : 2)) return ROIX_EINVAL;
    Layout L;
    if (!carve(ctx, g, &L, dtype)) return ROIX_ENOMEM;
    return enqueue_fused(lctx(ctx, stream), g, L, d_in, dtype, eb, crit, out);
}

roix_status roix_fused_background(roix_ctx* ctx, const float* d_in, roix_dims dims, const float* d_bg,
                                  int64_t bg_planes, roix_eb eb, const roix_criterion* crit,
                                  const roix_fused_out* out, float* d_work, void* stream) {
    Geom g;
    if (!ctx || !d_in || !d_bg || !d_work || !geom_of(dims, &g) || !eb_ok(eb) || !crit_ok(crit) || !out_ok(out, true))
        return ROIX_EINVAL;
    if (bg_planes != 1 && bg_planes != g.nz) return ROIX_EINVAL;
    if (!aligned(d_in, 4) || !aligned(d_bg, 4) || !aligned(d_work, 4)) return ROIX_EINVAL;
    // the workspace overlaps neither the image nor the reference
    const uintptr_t w0 = (uintptr_t)d_work, w1 = w0 + g.N * 4, i0 = (uintptr_t)d_in, i1 = i0 + g.N * 4;
    const uintptr_t b0 = (uintptr_t)d_bg, b1 = b0 + (size_t)bg_planes * (size_t)(g.nx * g.ny) * 4;
    if ((w0 < i1 && i0 < w1) || (w0 < b1 && b0 < w1)) return ROIX_EINVAL;
    Layout L;
    if (!carve(ctx, g, &L, ROIX_F32)) return ROIX_ENOMEM;
    const BgRef b = {d_bg, bg_planes == 1, d_work};
    return enqueue_fused_bg(lctx(ctx, stream), g, L, d_in, b, eb, crit, out);
}

roix_status roix_decode(roix_ctx* ctx, const roix_row* d_rows, int64_t rows_cap, const void* d_stream,
                        int64_t stream_cap_bytes, const float* d_outliers, int64_t outliers_cap,
                        const roix_quant_info* d_qinfo, const roix_extract_info* d_einfo, roix_dims dims,
                        float background, float* d_out, roix_decode_info* d_dinfo, void* stream) {
    Geom g;
    if (!ctx || !d_qinfo || !d_einfo || !d_out || !d_dinfo || !geom_of(dims, &g)) return ROIX_EINVAL;
    if (rows_cap < 0 || stream_cap_bytes < 0 || outliers_cap < 0) return ROIX_EINVAL;
    if ((rows_cap > 0 && (!d_rows || !aligned(d_rows, 8))) || (stream_cap_bytes > 0 && !d_stream) ||
        (outliers_cap > 0 && (!d_outliers || !aligned(d_outliers, 4))) || !aligned(d_out, 4) ||
        (d_stream && !aligned(d_stream, 4)) || !aligned(d_dinfo, 8))
        return ROIX_EINVAL;
    const size_t need = align256(sizeof(DevState)) + align256((size_t)g.nrows * 32);
    if (ctx->arena_bytes < need) return ROIX_ENOMEM;
    DevState* S = (DevState*)ctx->arena;
    uint4* desc = (uint4*)((uint8_t*)ctx->arena + align256(sizeof(DevState)));
    ROIX_TRY(launch_decode(lctx(ctx, stream), d_rows, (uint64_t)rows_cap, d_stream, (uint64_t)stream_cap_bytes,
                           d_outliers, (uint64_t)outliers_cap, d_qinfo, d_einfo, g, background, d_out, S, desc,
                           d_dinfo));
    return ROIX_OK;
}

roix_status roix_background(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, const float* d_bg,
                            int64_t bg_planes, roix_bg_op op, float* d_out, void* stream) {
    Geom g;
    if (!ctx || !d_in || !d_bg || !d_out || !geom_of(dims, &g)) return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (op != ROIX_BG_SUBTRACT && (op != ROIX_BG_ADD || dtype != ROIX_F32)) return ROIX_EINVAL;
    if (bg_planes != 1 && bg_planes != g.nz) return ROIX_EINVAL;
    const size_t es = dtype == ROIX_F32 ? 4 : 2;
    if (!aligned(d_in, es) || !aligned(d_bg, 4) || !aligned(d_out, 4)) return ROIX_EINVAL;
    // the output may be the float32 input itself, and must not overlap it otherwise
    const uintptr_t i0 = (uintptr_t)d_in, i1 = i0 + g.N * es, o0 = (uintptr_t)d_out, o1 = o0 + g.N * 4;
    if (!(dtype == ROIX_F32 && i0 == o0) && i0 < o1 && o0 < i1) return ROIX_EINVAL;
    const uintptr_t b0 = (uintptr_t)d_bg, b1 = b0 + (size_t)bg_planes * (size_t)(g.nx * g.ny) * 4;
    if (b0 < o1 && o0 < b1) return ROIX_EINVAL;
    ROIX_TRY(launch_background(lctx(ctx, stream), d_in, dtype, d_bg, bg_planes > 1, g, (int)op, d_out));
    return ROIX_OK;
}

size_t roix_abs_quantize_scratch_bytes(int64_t m) { return m < 0 ? 0 : absq_scratch_bytes(m); }

roix_status roix_abs_quantize(roix_ctx* ctx, const uint8_t* d_pixels, int64_t m, double e_abs, uint8_t* d_q,
                              roix_absq_info* d_info, void* stream) {
    if (!ctx || !d_info || m < 0 || !(e_abs >= 0.0) || !aligned(d_info, 8)) return ROIX_EINVAL;
    if (m > ((int64_t)1 << 40)) return ROIX_EINVAL;
    if (m > 0) {
        if (!d_pixels || !d_q || !aligned(d_pixels, 16) || !aligned(d_q, 16)) return ROIX_EINVAL;
        // apart: the output is written while later passes still read the pixels
        const uintptr_t a0 = (uintptr_t)d_pixels, b0 = (uintptr_t)d_q;
        if (a0 < b0 + (uint64_t)m && b0 < a0 + (uint64_t)m) return ROIX_EINVAL;
    }
    if (ctx->arena_bytes < absq_scratch_bytes(m)) return ROIX_ENOMEM;
    // integer pixels: |Q - D| <= E exactly when |Q - D| <= floor(E); groups span at most 2 floor(E)
    const double ef = e_abs >= 1024.0 ? 1024.0 : floor(e_abs);
    const uint32_t K = 2.0 * ef >= 255.0 ? 255u : (uint32_t)(2.0 * ef);
    ROIX_TRY(launch_absq(lctx(ctx, stream), d_pixels, m, K, d_q, ctx->arena, d_info));
    return ROIX_OK;
}

roix_status roix_section(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims,
                         const roix_fused_out* out, uint8_t* d_section, int64_t section_cap,
                         roix_section_info* d_info, void* stream) {
    Geom g;
    if (!ctx || !d_in || !out || !d_info || !geom_of(dims, &g) || section_cap < 0) return ROIX_EINVAL;
    if (dtype != ROIX_F32 && dtype != ROIX_U16) return ROIX_EINVAL;
    if (!aligned(d_in, dtype == ROIX_F32 ? 4 : 2) || !aligned(d_info, 8)) return ROIX_EINVAL;
    if (!out->d_qinfo || !out->d_einfo || !aligned(out->d_qinfo, 8) || !aligned(out->d_einfo, 8)) return ROIX_EINVAL;
    if (out->rows_cap < 0 || out->stream_cap_bytes < 0) return ROIX_EINVAL;
    if (out->rows_cap > 0 && (!out->d_rows || !aligned(out->d_rows, 8))) return ROIX_EINVAL;
    if (out->stream_cap_bytes > 0 && (!out->d_stream || !aligned(out->d_stream, 16))) return ROIX_EINVAL;
    if (section_cap > 0 && (!d_section || !aligned(d_section, 16))) return ROIX_EINVAL;
    if (ctx->arena_bytes < section_scratch_bytes()) return ROIX_ENOMEM;
    ROIX_TRY(launch_section(lctx(ctx, stream), d_in, dtype, g, out, d_section, section_cap, d_info, ctx->arena,
                            ctx->arena_bytes));
    return ROIX_OK;
}

static bool huff_n_ok(int64_t n) { return n >= 0 && n <= ((int64_t)1 << 40); }

roix_status roix_huff_encode(roix_ctx* ctx, const uint8_t* d_in, int64_t n, uint8_t* d_lengths,
                             uint64_t* d_block_off, uint16_t* d_sub_bits, uint32_t* d_payload,
                             int64_t payload_cap_words, roix_huff_info* d_info, void* stream) {
    if (!ctx || !d_lengths || !d_block_off || !d_info || !huff_n_ok(n) || payload_cap_words < 0) return ROIX_EINVAL;
    if (!aligned(d_block_off, 8) || !aligned(d_info, 8) || !aligned(d_sub_bits, 2)) return ROIX_EINVAL;
    if (n > 0 && (!d_in || !aligned(d_in, 16))) return ROIX_EINVAL;
    if (payload_cap_words > 0 && (!d_payload || !aligned(d_payload, 4))) return ROIX_EINVAL;
    if (ctx->arena_bytes < huff_scratch_bytes()) return ROIX_ENOMEM;
    ROIX_TRY(launch_huff_encode(lctx(ctx, stream), d_in, n, d_lengths, (unsigned long long*)d_block_off, d_sub_bits,
                                d_payload, payload_cap_words, ctx->arena, d_info));
    return ROIX_OK;
}

roix_status roix_huff_decode(roix_ctx* ctx, const uint8_t* d_lengths, const uint64_t* d_block_off,
                             const uint16_t* d_sub_bits, const uint32_t* d_payload, int64_t payload_words, int64_t n,
                             uint8_t* d_out, roix_huff_info* d_info, void* stream) {
    if (!ctx || !d_lengths || !d_block_off || !d_info || !huff_n_ok(n) || payload_words < 0) return ROIX_EINVAL;
    if (!aligned(d_block_off, 8) || !aligned(d_info, 8) || !aligned(d_sub_bits, 2)) return ROIX_EINVAL;
    if (n > 0 && (!d_out || !aligned(d_out, 16))) return ROIX_EINVAL;
    if (payload_words > 0 && (!d_payload || !aligned(d_payload, 4))) return ROIX_EINVAL;
    if (ctx->arena_bytes < huff_scratch_bytes()) return ROIX_ENOMEM;
    ROIX_TRY(launch_huff_decode(lctx(ctx, stream), d_lengths, (const unsigned long long*)d_block_off, d_sub_bits,
                                d_payload, payload_words, n, d_out, ctx->arena, d_info));
    return ROIX_OK;
}

roix_status roix_ctx_set_param(roix_ctx* ctx, const char* name, int64_t value) {
    if (!ctx || !name) return ROIX_EINVAL;
    const bool pos = value >= 1 && value <= (1 << 22);
    if (strcmp(name, "grid_stream") == 0 && pos) ctx->grid_stream = (int)value;
    else if (strcmp(name, "grid_read") == 0 && pos) ctx->grid_read = (int)value;
    else if (strcmp(name, "grid_emit") == 0 && pos) ctx->grid_emit = (int)value;
    else if (strcmp(name, "grid_mask") == 0 && pos) ctx->grid_mask = (int)value;
    else if (strcmp(name, "seg_grid") == 0 && pos) ctx->seg_grid = (int)value;
    else if (strcmp(name, "stats_grid") == 0 && pos) ctx->stats_grid = (int)value;
    else if (strcmp(name, "seg_runs") == 0 && value >= 0 && value <= 16384 && value % 256 == 0)
        ctx->seg_runs = (int)value;
    else if (strcmp(name, "batch_group") == 0 && value >= 0 && value <= (1 << 20)) ctx->batch_group = (int)value;
    else if (strcmp(name, "batch_lanes") == 0 && value >= 1 && value <= 4) ctx->batch_lanes = (int)value;
    else if (strcmp(name, "batch_fused16_min_voxels") == 0 && value >= 0 && value <= (1ll << 40))
        ctx->batch_p16_min = (uint64_t)value;
    else if (strcmp(name, "batch_graph") == 0 && (value == 0 || value == 1)) ctx->batch_graph = (int)value;
    else if (strcmp(name, "fused16_min_voxels") == 0 && value >= 0 && value <= (1ll << 40))
        ctx->p16_min = (uint64_t)value;
    else return ROIX_EINVAL;
    return ROIX_OK;
}

roix_status roix_ctx_get_param(roix_ctx* ctx, const char* name, int64_t* value) {
    if (!ctx || !name || !value) return ROIX_EINVAL;
    if (strcmp(name, "grid_stream") == 0) *value = ctx->grid_stream;
    else if (strcmp(name, "grid_read") == 0) *value = ctx->grid_read;
    else if (strcmp(name, "grid_emit") == 0) *value = ctx->grid_emit;
    else if (strcmp(name, "grid_mask") == 0) *value = ctx->grid_mask;
    else if (strcmp(name, "seg_grid") == 0) *value = ctx->seg_grid;
    else if (strcmp(name, "stats_grid") == 0) *value = ctx->stats_grid;
    else if (strcmp(name, "seg_runs") == 0) *value = ctx->seg_runs;
    else if (strcmp(name, "batch_group") == 0) *value = ctx->batch_group;
    else if (strcmp(name, "batch_lanes") == 0) *value = ctx->batch_lanes;
    else if (strcmp(name, "batch_fused16_min_voxels") == 0) *value = (int64_t)ctx->batch_p16_min;
    else if (strcmp(name, "batch_graph") == 0) *value = ctx->batch_graph;
    else if (strcmp(name, "compute_units") == 0) *value = ctx->cus;
    else if (strcmp(name, "fused16_min_voxels") == 0) *value = (int64_t)ctx->p16_min;
    else return ROIX_EINVAL;
    return ROIX_OK;
}

}  // extern "C"
