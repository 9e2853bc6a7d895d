// batch.hip - the batched form: many volumes of any shapes through the fused
// path with one launch per stage for all of them.
//
// Each volume's plain launch sequence is recorded (body, grid, arguments) on
// its own part of the arena; the voxel-proportional passes then split their
// grid among the volumes of each merged launch by voxels.  The sequences are merged: each step launches one body for
// every volume whose next launch it is, so each volume's launches keep their
// order and a batch takes about as many launches as one volume, whatever
// the number of volumes (per lane: the volumes are dealt out to lanes, by
// default two, whose sequences run concurrently on two streams).  The argument tables of all launches go to the
// device in one copy; the launch sequence is captured into a HIP graph and
// replayed while the batch's structure (bodies, grids, table offsets) is the
// same -- the buffers may change from call to call.
#include <algorithm>
#include <cmath>

#include <string.h>

#include "host.h"

using namespace roix;

void batch_destroy(BatchState& b) {
    if (b.exec) hipGraphExecDestroy(b.exec);
    if (b.graph) hipGraphDestroy(b.graph);
    if (b.ev_in) hipEventDestroy(b.ev_in);
    if (b.ev_out) hipEventDestroy(b.ev_out);
    if (b.ev_copy) hipEventDestroy(b.ev_copy);
    if (b.origin) hipStreamDestroy(b.origin);
    for (int l = 0; l < 3; ++l) {
        if (b.lane_stream[l]) hipStreamDestroy(b.lane_stream[l]);
        if (b.lane_done[l]) hipEventDestroy(b.lane_done[l]);
    }
    if (b.pinned) hipHostFree(b.pinned);
    b = BatchState();
}

namespace {

// one merged launch: body `fn` for the volumes in `who` (volume, index of the
// launch in its recorded sequence)
struct Merged {
    ManyLaunch fn;
    uint32_t block, shmem, arg_size, arg_align;
    std::vector<std::pair<int, size_t>> who;
    size_t args_off = 0, start_off = 0;
    uint32_t total = 0;
};

// The next launch of the volume with the most launches left, for every
// volume whose next launch is the same body: a shortest-common-supersequence
// heuristic that keeps the volumes in step.
void merge(const std::vector<Recorder>& rec, std::vector<Merged>& out) {
    const size_t n = rec.size();
    std::vector<size_t> pos(n, 0);
    while (true) {
        int pick = -1;
        size_t left = 0;
        for (size_t i = 0; i < n; ++i) {
            const size_t r = rec[i].seq.size() - pos[i];
            if (r > left) {
                left = r;
                pick = (int)i;
            }
        }
        if (pick < 0) break;
        const RecLaunch& h = rec[pick].seq[pos[pick]];
        Merged m;
        m.fn = h.launch;
        m.block = h.block;
        m.shmem = h.shmem;
        m.arg_size = h.arg_size;
        m.arg_align = h.arg_align;
        for (size_t i = 0; i < n; ++i) {
            if (pos[i] >= rec[i].seq.size()) continue;
            const RecLaunch& r = rec[i].seq[pos[i]];
            if (r.launch != m.fn || r.block != m.block || r.shmem != m.shmem || r.arg_size != m.arg_size) continue;
            m.who.emplace_back((int)i, pos[i]);
            ++pos[i];
        }
        out.push_back(std::move(m));
    }
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Arguments and workgroup prefix tables of the merged launches, appended to
// blob; false when a grid does not fit 32 bits.
bool pack(const std::vector<Recorder>& rec, std::vector<Merged>& ms, std::vector<uint8_t>& blob) {
    for (Merged& m : ms) {
        size_t o = round_up(blob.size(), std::max<size_t>(16, m.arg_align));
        m.args_off = o;
        blob.resize(o + (size_t)m.arg_size * m.who.size());
        for (size_t k = 0; k < m.who.size(); ++k) {
            const RecLaunch& r = rec[m.who[k].first].seq[m.who[k].second];
            memcpy(blob.data() + o + (size_t)m.arg_size * k, r.args.data(), m.arg_size);
        }
        o = round_up(blob.size(), 16);
        m.start_off = o;
        blob.resize(o + 4 * (m.who.size() + 2));
        uint64_t acc = 0;
        uint32_t* st = reinterpret_cast<uint32_t*>(blob.data() + o);
        for (size_t k = 0; k < m.who.size(); ++k) {
            st[k] = (uint32_t)acc;
            acc += rec[m.who[k].first].seq[m.who[k].second].grid;
            if (acc > 0x7FFFFFFFull) return false;
        }
        st[m.who.size()] = (uint32_t)acc;
        st[m.who.size() + 1] = kTableMark;
        m.total = (uint32_t)acc;
    }
    return true;
}

}  // namespace

struct BatchPlan {
    std::vector<uint8_t> key;
    std::vector<std::vector<Merged>> lanes;  // the merged launches of each lane, in order
};

namespace {

void issue(const std::vector<Merged>& ms, const uint8_t* dblob, hipStream_t s) {
    for (const Merged& m : ms)
        if (m.total)
            m.fn(dblob + m.args_off, reinterpret_cast<const uint32_t*>(dblob + m.start_off), (uint32_t)m.who.size(),
                 m.total, m.block, m.shmem, s);
}

roix_status ready(BatchState& b) {
    if (!b.ev_in && hipEventCreateWithFlags(&b.ev_in, hipEventDisableTiming) != hipSuccess) return ROIX_EDEVICE;
    if (!b.ev_out && hipEventCreateWithFlags(&b.ev_out, hipEventDisableTiming) != hipSuccess) return ROIX_EDEVICE;
    if (!b.ev_copy && hipEventCreateWithFlags(&b.ev_copy, hipEventDisableTiming) != hipSuccess) return ROIX_EDEVICE;
    if (!b.origin && hipStreamCreateWithFlags(&b.origin, hipStreamNonBlocking) != hipSuccess) return ROIX_EDEVICE;
    for (int l = 0; l < 3; ++l) {
        if (!b.lane_stream[l] && hipStreamCreateWithFlags(&b.lane_stream[l], hipStreamNonBlocking) != hipSuccess)
            return ROIX_EDEVICE;
        if (!b.lane_done[l] && hipEventCreateWithFlags(&b.lane_done[l], hipEventDisableTiming) != hipSuccess)
            return ROIX_EDEVICE;
    }
    return ROIX_OK;
}

}  // namespace

namespace {

// Record, merge and pack the batch into b.plan and the pinned tables.
roix_status plan_batch(roix_ctx* ctx, int32_t n, const roix_volume_desc* vols, const std::vector<Geom>& gs,
                       const std::vector<int>& kind, const std::vector<size_t>& need, size_t avail, size_t reserve,
                       const std::vector<uint8_t>& pkey) {
    BatchState& b = ctx->batch;
    uint8_t* const base = (uint8_t*)ctx->arena;
    hipStream_t stream = nullptr;  // recording launches nothing
    auto plan = std::make_shared<BatchPlan>();
    std::vector<uint8_t> blob;
    // Lanes: volume i goes to lane i mod nl, each lane with its own part of
    // the arena and its own launch sequence, the lanes running concurrently
    // (so that one lane's stages bound by a few volumes' runs leave the chip
    // to the other's).  One lane when the graph replays the batch or when a
    // volume's worst-case layout does not fit a part.
    int nl = ctx->batch_graph ? 1 : std::max(1, std::min<int>(ctx->batch_lanes, n));
    size_t part = nl > 1 ? (avail / (size_t)nl) & ~(size_t)255 : avail;
    for (int i = 0; i < n && nl > 1; ++i)
        if (align256(need[i]) > part) {
            nl = 1;
            part = avail;
        }
    plan->lanes.resize((size_t)nl);
    for (int l = 0; l < nl; ++l) {
        std::vector<Merged>& all = plan->lanes[(size_t)l];
        std::vector<int> idx;
        for (int i = l; i < n; i += nl) idx.push_back(i);
        const int m = (int)idx.size();
        uint8_t* const lbase = base + (size_t)l * part;
        // groups of consecutive volumes of the lane whose worst-case layouts fit
        // its part together (a volume too large for that gets the whole part alone)
        std::vector<std::pair<int, int>> groups;  // positions in idx
        for (int a = 0; a < m;) {
            int c = a;
            size_t used = 0;
            while (c < m && (c == a || used + align256(need[idx[c]]) <= part) &&
                   (ctx->batch_group <= 0 || c - a < ctx->batch_group)) {
                used += align256(need[idx[c]]);
                ++c;
            }
            groups.emplace_back(a, c);
            a = c;
        }

        for (const auto& gr : groups) {
            const int a0 = gr.first, a1 = gr.second;
            std::vector<Recorder> rec((size_t)(a1 - a0)), half((size_t)(a1 - a0));
            size_t off = 0;
            for (int a = a0; a < a1; ++a) {
                const int i = idx[a];
                const roix_volume_desc& d = vols[i];
                const size_t bytes = (a1 - a0 == 1) ? part : align256(need[i]);
                Layout L;
                int k = kind[i];
                if (a1 - a0 == 1) k = proxy_kind_for(gs[i], (roix_dtype)d.dtype, bytes, ctx->batch_p16_min);
                if (!carve_at(lbase + off, bytes, gs[i], &L, k)) return ROIX_ENOMEM;
                off += bytes;
                // the plain launch parameters, recorded twice: as they are, and
                // with the grids of the passes whose work follows the voxels
                // (range, quantise + histogram, mask words and runs) halved,
                // which tells those launches apart.  The others keep the plain
                // grid: their work follows runs, components or codes, which only
                // the device knows, and a volume of few voxels may hold many.
                for (int pass = 0; pass < 2; ++pass) {
                    LaunchCtx lc = lctx(ctx, stream);
                    lc.timer = nullptr;
                    lc.rec = pass == 0 ? &rec[(size_t)(a - a0)] : &half[(size_t)(a - a0)];
                    const double share = pass == 0 ? 1.0 : 0.5;
                    auto sc = [&](int v, int lo) {
                        const int s = (int)std::lround((double)v * share);
                        return std::max(lo, std::min(v, s));
                    };
                    lc.grid_read = sc(ctx->grid_read, 4);
                    lc.grid_mask = sc(ctx->grid_mask, 8);
                    lc.grid_vox = sc(ctx->grid_stream, 8);
                    const roix_status st =
                        enqueue_fused(lc, gs[i], L, d.d_in, (roix_dtype)d.dtype, d.eb, &d.crit, &d.out);
                    if (st != ROIX_OK) return st;
                    if (lc.rec->bad) return ROIX_EDEVICE;
                }
                if (half[(size_t)(a - a0)].seq.size() != rec[(size_t)(a - a0)].seq.size()) return ROIX_EDEVICE;
            }
            std::vector<Merged> ms;
            merge(rec, ms);
            // A merged launch of a voxel-proportional pass splits its plain grid
            // among its own volumes by their voxels (volumes of one group take
            // different kernels -- flows, row alignments -- so a share of the
            // whole group's voxels would leave each such launch part of the chip).
            for (const Merged& m : ms) {
                bool prop = false;
                uint32_t cap = 0;
                double nsum = 0.0;
                for (const auto& w : m.who) {
                    const uint32_t g = rec[(size_t)w.first].seq[w.second].grid;
                    prop = prop || half[(size_t)w.first].seq[w.second].grid < g;
                    cap = std::max(cap, g);
                    nsum += (double)gs[idx[a0 + w.first]].N;
                }
                if (!prop || nsum <= 0.0) continue;
                for (const auto& w : m.who) {
                    uint32_t& g = rec[(size_t)w.first].seq[w.second].grid;
                    const double want = std::round((double)cap * (double)gs[idx[a0 + w.first]].N / nsum);
                    g = std::min(g, std::max<uint32_t>(std::min<uint32_t>(g, 8u), (uint32_t)want));
                }
            }
            if (!pack(rec, ms, blob)) return ROIX_EINVAL;
            all.insert(all.end(), ms.begin(), ms.end());
        }
    }
    if (blob.size() > reserve) return ROIX_ENOMEM;
    // the tables go through pinned memory: an asynchronous copy from
    // pageable memory may have the runtime pin the caller's pages, which a
    // host can refuse (the copy would then not happen); the previous copy
    // must have read the buffer before it changes
    if (hipEventSynchronize(b.ev_copy) != hipSuccess) return ROIX_EDEVICE;
    if (b.pinned_cap < blob.size()) {
        if (b.pinned) hipHostFree(b.pinned);
        b.pinned = nullptr;
        b.pinned_cap = 0;
        const size_t cap = round_up(std::max<size_t>(blob.size(), (size_t)1 << 20), (size_t)1 << 16);
        if (hipHostMalloc((void**)&b.pinned, cap, hipHostMallocDefault) != hipSuccess) {
            b.pinned = nullptr;
            b.plan.reset();
            return ROIX_ENOMEM;
        }
        b.pinned_cap = cap;
    }
    memcpy(b.pinned, blob.data(), blob.size());
    b.pinned_bytes = blob.size();
    plan->key = pkey;
    b.plan = plan;
    return ROIX_OK;
}

}  // namespace

extern "C" roix_status roix_fused_batch(roix_ctx* ctx, int32_t n, const roix_volume_desc* vols, void* stream_) {
    if (!ctx || n < 0 || (n > 0 && !vols)) return ROIX_EINVAL;
    if (n == 0) return ROIX_OK;
    std::vector<Geom> gs(n);
    std::vector<int> kind(n);
    std::vector<size_t> need(n);
    for (int i = 0; i < n; ++i) {
        const roix_volume_desc& d = vols[i];
        if (!d.d_in || !geom_of(d.dims, &gs[i]) || !eb_ok(d.eb) || !crit_ok(&d.crit) || !out_ok(&d.out, true))
            return ROIX_EINVAL;
        if (d.dtype != ROIX_F32 && d.dtype != ROIX_U16) return ROIX_EINVAL;
        if (!aligned(d.d_in, d.dtype == ROIX_F32 ? 4 : 2)) return ROIX_EINVAL;
        kind[i] = proxy_kind(gs[i], (roix_dtype)d.dtype, ctx->batch_p16_min);
        need[i] = fixed_bytes(gs[i], kind[i]) + (size_t)worst_runs(gs[i]) * kRunBytes;
    }
    // the argument tables live at the end of the arena, from a 256-byte
    // boundary (the arena's size need not be a multiple of anything)
    const size_t reserve = round_up(std::min<size_t>(ctx->arena_bytes / 4, (size_t)65536 + (size_t)n * 65536), 256);
    if (ctx->arena_bytes < reserve + 4096) return ROIX_ENOMEM;
    const size_t avail = (ctx->arena_bytes - reserve) & ~(size_t)255;
    uint8_t* const base = (uint8_t*)ctx->arena;
    uint8_t* const dblob = base + avail;
    hipStream_t stream = (hipStream_t)stream_;
    BatchState& b = ctx->batch;
    if (ready(b) != ROIX_OK) return ROIX_EDEVICE;
    // the tables depend only on the descriptors, the arena and the parameters
    std::vector<uint8_t> pkey;
    {
        auto put = [&](const void* p, size_t k) { pkey.insert(pkey.end(), (const uint8_t*)p, (const uint8_t*)p + k); };
        put(vols, sizeof(roix_volume_desc) * (size_t)n);
        const int64_t prm[14] = {(int64_t)(uintptr_t)ctx->arena, (int64_t)ctx->arena_bytes, ctx->grid_stream,
                                 ctx->grid_read, ctx->grid_emit, ctx->grid_mask, ctx->seg_grid, ctx->seg_runs,
                                 ctx->stats_grid, (int64_t)ctx->p16_min, (int64_t)ctx->batch_p16_min,
                                 ctx->batch_group, ctx->batch_lanes, ctx->batch_graph};
        put(prm, sizeof prm);
    }
    if (!b.plan || b.plan->key != pkey) {
        const roix_status st = plan_batch(ctx, n, vols, gs, kind, need, avail, reserve, pkey);
        if (st != ROIX_OK) return st;
    }
    const std::vector<std::vector<Merged>>& lanes = b.plan->lanes;
    // the tables go to the device on every call: plain calls between two
    // batches may have used the end of the arena
    ROIX_TRY(hipMemcpyAsync(dblob, b.pinned, b.pinned_bytes, hipMemcpyHostToDevice, stream));
    ROIX_TRY(hipEventRecord(b.ev_copy, stream));
    if (!ctx->batch_graph) {
        // lane 0 on the caller's stream, the others on the context's lane
        // streams from the tables' copy on, the caller's stream waiting for
        // every lane at the end
        const int nl = (int)lanes.size();
        if (nl > 1) ROIX_TRY(hipEventRecord(b.ev_in, stream));
        for (int l = 1; l < nl; ++l) ROIX_TRY(hipStreamWaitEvent(b.lane_stream[l - 1], b.ev_in, 0));
        for (int l = 0; l < nl; ++l) issue(lanes[(size_t)l], dblob, l == 0 ? stream : b.lane_stream[l - 1]);
        ROIX_TRY(hipGetLastError());
        for (int l = 1; l < nl; ++l) {
            ROIX_TRY(hipEventRecord(b.lane_done[l - 1], b.lane_stream[l - 1]));
            ROIX_TRY(hipStreamWaitEvent(stream, b.lane_done[l - 1], 0));
        }
        return ROIX_OK;
    }
    const std::vector<Merged>& all = lanes[0];  // one lane under the graph
    // the graph depends on the bodies, grids and table offsets only
    std::vector<uint8_t> key;
    auto put = [&](const void* p, size_t k) { key.insert(key.end(), (const uint8_t*)p, (const uint8_t*)p + k); };
    const uintptr_t db = (uintptr_t)dblob;
    put(&db, sizeof db);
    for (const Merged& m : all) {
        const uint64_t f[6] = {(uint64_t)(uintptr_t)m.fn, m.block,          m.shmem,
                               m.who.size(),               m.args_off,       m.start_off};
        put(f, sizeof f);
        put(&m.total, sizeof m.total);
    }
    if (!b.exec || b.key != key) {
        if (b.exec) hipGraphExecDestroy(b.exec);
        if (b.graph) hipGraphDestroy(b.graph);
        b.exec = nullptr;
        b.graph = nullptr;
        b.key.clear();
        // captured on the context's own stream (the caller's may be the
        // legacy default stream, which cannot be captured)
        ROIX_TRY(hipStreamBeginCapture(b.origin, hipStreamCaptureModeThreadLocal));
        issue(all, dblob, b.origin);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(b.origin, &graph);
        (void)hipGetLastError();
        if (e != hipSuccess || !graph) return ROIX_EDEVICE;
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(graph);
            return ROIX_EDEVICE;
        }
        b.graph = graph;
        b.exec = exec;
        b.key = key;
    }
    ROIX_TRY(hipEventRecord(b.ev_in, stream));
    ROIX_TRY(hipStreamWaitEvent(b.origin, b.ev_in, 0));
    ROIX_TRY(hipGraphLaunch(b.exec, b.origin));
    ROIX_TRY(hipEventRecord(b.ev_out, b.origin));
    ROIX_TRY(hipStreamWaitEvent(stream, b.ev_out, 0));
    return ROIX_OK;
}
