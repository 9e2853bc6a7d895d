// k_label.hip - binary mask, foreground runs, 3-D connected components of the
// runs, per-component statistics and the keep rule.
//
// The mask (object = proxy byte above the threshold byte) is turned into a
// row bitmask with one wave ballot per 64 voxels, and every row (z, y) into
// its maximal runs of object voxels.  Runs are numbered in raster order, so
// the run with the smallest number of a component holds the component's
// smallest linear voxel index.  Runs of neighbouring rows that touch are
// united with a lock-free union-find that always links the larger root under
// the smaller one; after flattening, the root of a component is its first run
// and the canonical label is that run's first voxel.  Work is O(runs), not
// O(voxels): per-voxel traffic is one read of the 1-byte proxy and one
// write + read of the 1-bit mask.
#include "common.h"

namespace roix {

__device__ __forceinline__ bool block_exit_l(const DevState* S) {
    __shared__ int s_exit;
    if (threadIdx.x == 0) s_exit = __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    return s_exit != 0;
}

__device__ __forceinline__ bool thread_exit(const DevState* S) {
    return __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

static int grid_for(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------------- mask bits + counts

// One wave per row: lane l reads proxy byte 64*w + l; the ballot of
// (byte > threshold) is mask word w.  Run starts are 1-bits whose left
// neighbour is 0.  Words are staged one per lane and stored 64 at a time.
__global__ __launch_bounds__(kBlock) void k_mask_runs(const uint8_t* __restrict__ proxy, int64_t nx, int64_t nrows,
                                                      int64_t W, DevState* S, uint64_t* __restrict__ maskbits,
                                                      uint32_t* __restrict__ row_nruns) {
    if (block_exit_l(S)) return;
    const int thr = S->proxy_thr;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    unsigned long long nmask = 0;
    constexpr int kB = 8;
    for (int64_t row = wave; row < nrows; row += nwaves) {
        const uint8_t* p = proxy + row * nx;
        uint64_t* mb = maskbits + row * W;
        uint64_t carry = 0, myword = 0;
        uint32_t runs = 0;
        for (int64_t w0 = 0; w0 < W; w0 += kB) {
            uint32_t b[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                int64_t x = (w0 + k) * 64 + lane;
                b[k] = (x < nx) ? (uint32_t)p[x] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int64_t w = w0 + k;
                if (w >= W) break;
                uint64_t m = __ballot((int)b[k] > thr);
                uint64_t starts = m & ~((m << 1) | carry);
                runs += (uint32_t)__popcll(starts);
                nmask += (unsigned long long)__popcll(m);
                carry = m >> 63;
                if ((w & 63) == lane) myword = m;
                if ((w & 63) == 63 || w == W - 1) {
                    int64_t idx = (w & ~(int64_t)63) + lane;
                    if (idx <= w) mb[idx] = myword;
                }
            }
        }
        if (lane == 0) row_nruns[row] = runs;
    }
    // nmask is wave-uniform: count it once per wave
    __shared__ unsigned long long s_n[kBlock / kWave];
    if (lane == 0) s_n[threadIdx.x / kWave] = nmask;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t += s_n[k];
        if (t) atomicAdd(&S->n_mask, t);
    }
}

hipError_t launch_mask_runs(const LaunchCtx& lc, const Geom& g, const Layout& L) {
    timer_begin(lc.timer, ST_MASK_RUNS, lc.stream);
    int grid = grid_for(g.nrows, kBlock / kWave, 8192);
    hipLaunchKernelGGL(k_mask_runs, dim3(grid), dim3(kBlock), 0, lc.stream, (const uint8_t*)L.proxy, g.nx, g.nrows,
                       g.W, L.S, L.maskbits, L.row_nruns);
    timer_end(lc.timer, ST_MASK_RUNS, lc.stream);
    return hipGetLastError();
}

// ----------------------------------------------------------------- runs

// One thread per row: walk the row's words; a start event opens a run, an
// end event (0-bit after a 1-bit) closes it.  parent[] starts as identity.
__global__ __launch_bounds__(kBlock) void k_runs_write(const uint64_t* __restrict__ maskbits, int64_t nrows, int64_t W,
                                                       const uint32_t* __restrict__ run_off, uint32_t* __restrict__ xs_out,
                                                       uint32_t* __restrict__ xe_out, uint32_t* __restrict__ parent,
                                                       const DevState* S) {
    if (thread_exit(S)) return;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < nrows; row += nthreads) {
        const uint64_t* mb = maskbits + row * W;
        uint32_t k = run_off[row];
        uint64_t carry = 0;
        uint32_t xs = 0;
        for (int64_t w = 0; w < W; ++w) {
            const uint64_t m = mb[w];
            const uint64_t prev = (m << 1) | carry;
            const uint64_t starts = m & ~prev;
            uint64_t ev = starts | (~m & prev);
            while (ev) {
                const int i = __ffsll((unsigned long long)ev) - 1;
                ev &= ev - 1;
                const uint32_t pos = (uint32_t)(w * 64 + i);
                if ((starts >> i) & 1ull) {
                    xs = pos;
                } else {
                    xs_out[k] = xs;
                    xe_out[k] = pos;
                    parent[k] = k;
                    ++k;
                }
            }
            carry = m >> 63;
        }
        if (carry) {
            xs_out[k] = xs;
            xe_out[k] = (uint32_t)(W * 64);
            parent[k] = k;
        }
    }
}

hipError_t launch_runs_write(const LaunchCtx& lc, const Geom& g, const Layout& L) {
    timer_begin(lc.timer, ST_RUNS, lc.stream);
    hipLaunchKernelGGL(k_runs_write, dim3(grid_for(g.nrows, kBlock, 16384)), dim3(kBlock), 0, lc.stream,
                       (const uint64_t*)L.maskbits, g.nrows, g.W, (const uint32_t*)L.run_off, L.run_xs, L.run_xe,
                       L.parent, (const DevState*)L.S);
    timer_end(lc.timer, ST_RUNS, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------ union-find

// Root of x with path halving.  Parent pointers only ever point to smaller
// run numbers, so the walk terminates; a halving store only writes an
// ancestor, which is safe against concurrent links (links only change roots).
__device__ __forceinline__ uint32_t find_root(uint32_t* parent, uint32_t x) {
    while (true) {
        uint32_t p = ld_relaxed(&parent[x]);
        if (p == x) return x;
        uint32_t gp = ld_relaxed(&parent[p]);
        if (gp == p) return p;
        st_relaxed(&parent[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void unite(uint32_t* parent, uint32_t a, uint32_t b) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    while (a != b) {
        if (a > b) {
            uint32_t t = a;
            a = b;
            b = t;
        }
        // link the larger root under the smaller one
        uint32_t old = atomicCAS(&parent[b], b, a);
        if (old == b) return;
        b = find_root(parent, old);
        a = find_root(parent, a);
    }
}

// Runs of rows r and rn (a neighbouring row) are connected when their x
// intervals overlap (6-connectivity) or touch within one voxel (26).
template <bool C26>
__device__ __forceinline__ void merge_rows(uint32_t* parent, const uint32_t* xs, const uint32_t* xe, uint32_t a,
                                           uint32_t a1, uint32_t b, uint32_t b1) {
    while (a < a1 && b < b1) {
        const uint32_t as = xs[a], ae = xe[a], bs = xs[b], be = xe[b];
        const bool hit = C26 ? (as <= be && bs <= ae) : (as < be && bs < ae);
        if (hit) unite(parent, a, b);
        if (ae < be)
            ++a;
        else if (be < ae)
            ++b;
        else {
            ++a;
            ++b;
        }
    }
}

// One thread per row (z, y): unite with the earlier neighbour rows
// (z, y-1), (z-1, y), and for 26-connectivity (z-1, y-1), (z-1, y+1).
template <bool C26>
__global__ __launch_bounds__(kBlock) void k_union(const uint32_t* __restrict__ run_off, const uint32_t* __restrict__ xs,
                                                  const uint32_t* __restrict__ xe, uint32_t* parent, int64_t ny,
                                                  int64_t nrows, const DevState* S) {
    if (thread_exit(S)) return;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += nthreads) {
        const uint32_t a0 = run_off[r], a1 = run_off[r + 1];
        if (a0 == a1) continue;
        const int64_t z = r / ny, y = r - z * ny;
        if (y > 0) merge_rows<C26>(parent, xs, xe, a0, a1, run_off[r - 1], run_off[r]);
        if (z > 0) {
            const int64_t rz = r - ny;
            merge_rows<C26>(parent, xs, xe, a0, a1, run_off[rz], run_off[rz + 1]);
            if (C26) {
                if (y > 0) merge_rows<C26>(parent, xs, xe, a0, a1, run_off[rz - 1], run_off[rz]);
                if (y < ny - 1) merge_rows<C26>(parent, xs, xe, a0, a1, run_off[rz + 1], run_off[rz + 2]);
            }
        }
    }
}

hipError_t launch_union(const LaunchCtx& lc, const Geom& g, const Layout& L, int conn) {
    timer_begin(lc.timer, ST_UNION, lc.stream);
    dim3 grid(grid_for(g.nrows, kBlock, 16384));
    if (conn == 26)
        hipLaunchKernelGGL(k_union<true>, grid, dim3(kBlock), 0, lc.stream, (const uint32_t*)L.run_off,
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, L.parent, g.ny, g.nrows,
                           (const DevState*)L.S);
    else
        hipLaunchKernelGGL(k_union<false>, grid, dim3(kBlock), 0, lc.stream, (const uint32_t*)L.run_off,
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, L.parent, g.ny, g.nrows,
                           (const DevState*)L.S);
    timer_end(lc.timer, ST_UNION, lc.stream);
    return hipGetLastError();
}

// Full compression: parent[i] = root(i); root flags for the component scan.
// The walk only reads: a halving store by one thread could otherwise put an
// intermediate ancestor back into an entry another thread has already set to
// its root.  Each entry is written by its own thread only, so every entry
// ends at its root.
__global__ __launch_bounds__(kBlock) void k_flatten(uint32_t* parent, uint32_t* root_flag, const DevState* S) {
    if (thread_exit(S)) return;
    const uint32_t n = S->n_runs;
    const uint32_t nthreads = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nthreads) {
        uint32_t r = i, p = ld_relaxed(&parent[i]);
        while (p != r) {
            r = p;
            p = ld_relaxed(&parent[r]);
        }
        st_relaxed(&parent[i], r);
        root_flag[i] = (r == i) ? 1u : 0u;
    }
}

hipError_t launch_flatten(const LaunchCtx& lc, const Layout& L) {
    timer_begin(lc.timer, ST_FLATTEN, lc.stream);
    hipLaunchKernelGGL(k_flatten, dim3(2048), dim3(kBlock), 0, lc.stream, L.parent, L.comp_id,
                       (const DevState*)L.S);
    timer_end(lc.timer, ST_FLATTEN, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------- component stats

constexpr int kRowsPerThread = 4;
constexpr int kSlots = 8;

struct Acc {
    unsigned long long size;
    uint32_t x0, x1, y0, y1, z0, z1;
};

__device__ __forceinline__ void acc_reset(Acc& a) {
    a.size = 0;
    a.x0 = a.y0 = a.z0 = 0xFFFFFFFFu;
    a.x1 = a.y1 = a.z1 = 0u;
}

__device__ __forceinline__ void acc_flush_global(roix_component* comps, uint32_t cid, const Acc& a) {
    roix_component* c = comps + cid;
    atomicAdd((unsigned long long*)&c->size, a.size);
    atomicMin(&c->x0, a.x0);
    atomicMax(&c->x1, a.x1);
    atomicMin(&c->y0, a.y0);
    atomicMax(&c->y1, a.y1);
    atomicMin(&c->z0, a.z0);
    atomicMax(&c->z1, a.z1);
}

// One thread per row: the entry of every component whose root run lies in
// the row (label = first voxel of the root run).
__global__ __launch_bounds__(kBlock) void k_comp_init(const uint32_t* __restrict__ run_off,
                                                      const uint32_t* __restrict__ xs, const uint32_t* parent,
                                                      const uint32_t* __restrict__ comp_id, int64_t nx, int64_t nrows,
                                                      roix_component* comps, const DevState* S) {
    if (thread_exit(S)) return;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += nthreads) {
        for (uint32_t i = run_off[r]; i < run_off[r + 1]; ++i) {
            if (parent[i] != i) continue;
            roix_component* c = comps + comp_id[i];
            c->label = (uint64_t)r * (uint64_t)nx + xs[i];
            c->size = 0;
            c->x0 = c->y0 = c->z0 = 0xFFFFFFFFu;
            c->x1 = c->y1 = c->z1 = 0u;
            c->kept = 0u;
            c->pad = 0u;
        }
    }
}

// Per-thread accumulation over kRowsPerThread rows, then a small LDS table of
// kSlots roots per workgroup so that a giant component costs one set of
// global atomics per workgroup instead of one per run.
__global__ __launch_bounds__(kBlock) void k_comp_stats(const uint32_t* __restrict__ run_off,
                                                       const uint32_t* __restrict__ xs, const uint32_t* __restrict__ xe,
                                                       const uint32_t* __restrict__ parent,
                                                       const uint32_t* __restrict__ comp_id, int64_t ny, int64_t nrows,
                                                       roix_component* comps, const DevState* S) {
    __shared__ uint32_t s_root[kSlots];
    __shared__ unsigned long long s_size[kSlots];
    __shared__ uint32_t s_bb[kSlots][6];
    if (threadIdx.x < kSlots) {
        s_root[threadIdx.x] = kNone;
        s_size[threadIdx.x] = 0;
        s_bb[threadIdx.x][0] = s_bb[threadIdx.x][2] = s_bb[threadIdx.x][4] = 0xFFFFFFFFu;
        s_bb[threadIdx.x][1] = s_bb[threadIdx.x][3] = s_bb[threadIdx.x][5] = 0u;
    }
    if (block_exit_l(S)) return;
    uint32_t cur = kNone;
    Acc a;
    acc_reset(a);
    const int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRowsPerThread;
    for (int rr = 0; rr < kRowsPerThread; ++rr) {
        const int64_t r = r0 + rr;
        if (r >= nrows) break;
        const uint32_t z = (uint32_t)(r / ny), y = (uint32_t)(r - (int64_t)z * ny);
        for (uint32_t i = run_off[r]; i < run_off[r + 1]; ++i) {
            const uint32_t root = parent[i];
            if (root != cur) {
                if (cur != kNone) acc_flush_global(comps, comp_id[cur], a);
                cur = root;
                acc_reset(a);
            }
            const uint32_t s = xs[i], e = xe[i];
            a.size += e - s;
            a.x0 = s < a.x0 ? s : a.x0;
            a.x1 = e > a.x1 ? e : a.x1;
            a.y0 = y < a.y0 ? y : a.y0;
            a.y1 = y + 1 > a.y1 ? y + 1 : a.y1;
            a.z0 = z < a.z0 ? z : a.z0;
            a.z1 = z + 1 > a.z1 ? z + 1 : a.z1;
        }
    }
    if (cur != kNone) {
        int slot = -1;
        const uint32_t h = cur % kSlots;
        for (int pr = 0; pr < kSlots; ++pr) {
            const uint32_t sl = (h + pr) % kSlots;
            const uint32_t old = atomicCAS(&s_root[sl], kNone, cur);
            if (old == kNone || old == cur) {
                slot = (int)sl;
                break;
            }
        }
        if (slot >= 0) {
            atomicAdd(&s_size[slot], a.size);
            atomicMin(&s_bb[slot][0], a.x0);
            atomicMax(&s_bb[slot][1], a.x1);
            atomicMin(&s_bb[slot][2], a.y0);
            atomicMax(&s_bb[slot][3], a.y1);
            atomicMin(&s_bb[slot][4], a.z0);
            atomicMax(&s_bb[slot][5], a.z1);
        } else {
            acc_flush_global(comps, comp_id[cur], a);
        }
    }
    __syncthreads();
    if (threadIdx.x < kSlots && s_root[threadIdx.x] != kNone) {
        Acc t;
        t.size = s_size[threadIdx.x];
        t.x0 = s_bb[threadIdx.x][0];
        t.x1 = s_bb[threadIdx.x][1];
        t.y0 = s_bb[threadIdx.x][2];
        t.y1 = s_bb[threadIdx.x][3];
        t.z0 = s_bb[threadIdx.x][4];
        t.z1 = s_bb[threadIdx.x][5];
        acc_flush_global(comps, comp_id[s_root[threadIdx.x]], t);
    }
}

hipError_t launch_comp_stats(const LaunchCtx& lc, const Geom& g, const Layout& L, roix_component* comps) {
    timer_begin(lc.timer, ST_COMPS, lc.stream);
    hipLaunchKernelGGL(k_comp_init, dim3(grid_for(g.nrows, kBlock, 16384)), dim3(kBlock), 0, lc.stream,
                       (const uint32_t*)L.run_off, (const uint32_t*)L.run_xs, (const uint32_t*)L.parent,
                       (const uint32_t*)L.comp_id, g.nx, g.nrows, comps, (const DevState*)L.S);
    int64_t per_block = (int64_t)kBlock * kRowsPerThread;
    int64_t grid = (g.nrows + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_comp_stats, dim3((unsigned)(grid < 1 ? 1 : grid)), dim3(kBlock), 0, lc.stream,
                       (const uint32_t*)L.run_off, (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe,
                       (const uint32_t*)L.parent, (const uint32_t*)L.comp_id, g.ny, g.nrows, comps,
                       (const DevState*)L.S);
    timer_end(lc.timer, ST_COMPS, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------- keep rule

__global__ __launch_bounds__(kBlock) void k_largest_max(const roix_component* comps, DevState* S) {
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_comps;
    unsigned long long m = 0;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        m = comps[c].size > m ? comps[c].size : m;
    m = wave_max(m);
    if (threadIdx.x % kWave == 0 && m) atomicMax(&S->max_size, m);
}

__global__ __launch_bounds__(kBlock) void k_largest_arg(const roix_component* comps, DevState* S) {
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_comps;
    const unsigned long long m = S->max_size;
    uint32_t best = kNone;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        if (comps[c].size == m && c < best) best = c;
    best = wave_min(best);
    if (threadIdx.x % kWave == 0 && best != kNone) atomicMin(&S->largest_cid, best);
}

// kept flags, counts and the union box of kept components
__global__ __launch_bounds__(kBlock) void k_keep_apply(roix_component* comps, uint8_t* kept_flag, int largest,
                                                       unsigned long long min_size, DevState* S) {
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_comps;
    const uint32_t lc = S->largest_cid;
    unsigned long long nk = 0, nv = 0;
    uint32_t bb[6] = {0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        roix_component* e = comps + c;
        const bool k = largest ? (c == lc) : (e->size >= min_size);
        e->kept = k ? 1u : 0u;
        kept_flag[c] = k ? 1 : 0;
        if (k) {
            nk += 1;
            nv += e->size;
            bb[0] = e->x0 < bb[0] ? e->x0 : bb[0];
            bb[1] = e->x1 > bb[1] ? e->x1 : bb[1];
            bb[2] = e->y0 < bb[2] ? e->y0 : bb[2];
            bb[3] = e->y1 > bb[3] ? e->y1 : bb[3];
            bb[4] = e->z0 < bb[4] ? e->z0 : bb[4];
            bb[5] = e->z1 > bb[5] ? e->z1 : bb[5];
        }
    }
    nk = wave_sum(nk);
    nv = wave_sum(nv);
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
        bb[k] = wave_min(bb[k]);
        bb[k + 1] = wave_max(bb[k + 1]);
    }
    if (threadIdx.x % kWave == 0 && nk) {
        atomicAdd(&S->n_kept, nk);
        atomicAdd(&S->n_kept_voxels, nv);
        atomicMin(&S->bbox[0], bb[0]);
        atomicMax(&S->bbox[1], bb[1]);
        atomicMin(&S->bbox[2], bb[2]);
        atomicMax(&S->bbox[3], bb[3]);
        atomicMin(&S->bbox[4], bb[4]);
        atomicMax(&S->bbox[5], bb[5]);
    }
}

hipError_t launch_keep(const LaunchCtx& lc, const Layout& L, roix_component* comps, const roix_criterion* crit) {
    timer_begin(lc.timer, ST_KEEP, lc.stream);
    const int largest = crit->keep == ROIX_KEEP_LARGEST;
    const int grid = 512;
    if (largest) {
        hipLaunchKernelGGL(k_largest_max, dim3(grid), dim3(kBlock), 0, lc.stream, (const roix_component*)comps, L.S);
        hipLaunchKernelGGL(k_largest_arg, dim3(grid), dim3(kBlock), 0, lc.stream, (const roix_component*)comps, L.S);
    }
    hipLaunchKernelGGL(k_keep_apply, dim3(grid), dim3(kBlock), 0, lc.stream, comps, L.kept_flag, largest,
                       (unsigned long long)(crit->min_size > 0 ? crit->min_size : 1), L.S);
    timer_end(lc.timer, ST_KEEP, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------- per-voxel keep / labels

// One wave per row: lane x finds the run containing x (if any) by walking the
// row's runs in order; keep = the component's flag, label = its label.
__global__ __launch_bounds__(kBlock) void k_voxel_out(const uint32_t* __restrict__ run_off,
                                                      const uint32_t* __restrict__ xs, const uint32_t* __restrict__ xe,
                                                      const uint32_t* __restrict__ parent,
                                                      const uint32_t* __restrict__ comp_id,
                                                      const uint8_t* __restrict__ kept_flag,
                                                      const roix_component* __restrict__ comps, int64_t nx,
                                                      int64_t nrows, uint8_t* keep, int64_t* labels,
                                                      const DevState* S) {
    if (thread_exit(S)) return;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = wave; r < nrows; r += nwaves) {
        const uint32_t a1 = run_off[r + 1];
        uint32_t j = run_off[r];
        for (int64_t x0 = 0; x0 < nx; x0 += kWave) {
            const int64_t x = x0 + lane;
            if (x >= nx) break;
            while (j < a1 && (int64_t)xe[j] <= x) ++j;
            const bool in = j < a1 && (int64_t)xs[j] <= x;
            uint8_t k = 0;
            int64_t lab = -1;
            if (in) {
                const uint32_t cid = comp_id[parent[j]];
                k = kept_flag[cid];
                lab = (int64_t)comps[cid].label;
            }
            const uint64_t v = (uint64_t)r * (uint64_t)nx + (uint64_t)x;
            keep[v] = k;
            if (labels) labels[v] = lab;
        }
    }
}

hipError_t launch_voxel_out(const LaunchCtx& lc, const Geom& g, const Layout& L, const roix_component* comps,
                            uint8_t* keep, int64_t* labels) {
    timer_begin(lc.timer, ST_VOXEL_OUT, lc.stream);
    hipLaunchKernelGGL(k_voxel_out, dim3(grid_for(g.nrows, kBlock / kWave, 16384)), dim3(kBlock), 0, lc.stream,
                       (const uint32_t*)L.run_off, (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe,
                       (const uint32_t*)L.parent, (const uint32_t*)L.comp_id, (const uint8_t*)L.kept_flag, comps,
                       g.nx, g.nrows, keep, labels, (const DevState*)L.S);
    timer_end(lc.timer, ST_VOXEL_OUT, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
