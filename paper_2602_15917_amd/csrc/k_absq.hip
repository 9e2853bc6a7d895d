// k_absq.hip - the paper's absolute error-bounded quantisation of an 8-bit
// pixel sequence (Sec. 4.2.3): groups grow while the intervals
// [D - E, D + E] of their pixels intersect, i.e. while max - min <= 2E over
// the group, and every pixel of a group is written as floor((min + max) / 2)
// (the floored midpoint of the intersection), clipped to 0..255.  On integer
// pixels the tolerance is floor(E).
//
// The scan is sequential: where a group starts depends on where the one
// before it started.  Here the sequence is cut into chunks of 256 pixels, one
// chunk per lane, and:
//  1. speculation: every chunk is scanned as if a group started at its first
//     pixel; its group starts (a bit per pixel) and the group left open at
//     its end (min, max, first pixel) are kept;
//  2. rounds: every chunk is scanned again from the open group its
//     predecessor left in the previous round, until a group starts where a
//     speculative one does: from there the two chains are the same, so the
//     rest is the speculation's.  The true chain and the speculative one
//     interleave and almost always meet within a few groups.  The rescan
//     also gives the value of the entering group when it ends in the chunk.
//     A chunk whose entry did not change keeps its result; one round usually
//     settles every chunk and a second finds nothing to change.  After
//     kAqRounds rounds a chunk whose predecessor still changed is settled by
//     a one-wave sequential pass (sequences whose chains never meet, such as
//     long exact ramps);
//  3. the value of every group that crosses a chunk end goes, from the chunk
//     where the group ends, into a slot of the chunk where it starts;
//  4. the speculation already wrote its own groups' values (the running
//     value of the open group kept at its first pixel in LDS, spread by a
//     second sweep, the tile stored); every chunk is rescanned from its
//     settled entry up to where its true chain meets the speculative one,
//     the bytes before that point rewritten with the true groups' values and
//     the group crossing the chunk end given its slot's value.
// Chunks of a wave are staged through LDS as a 16 KB tile, loaded and stored
// with coalesced 16-byte accesses; each chunk's 64 words are padded to 65 so
// that the lanes' word-by-word reads fall in distinct banks.
#include "common.h"

namespace roix {

constexpr int kAqC = 256;                 // pixels per chunk (one lane)
constexpr int kAqWords = kAqC / 4;        // 32-bit words per chunk
constexpr int kAqStride = kAqWords + 1;   // LDS words per chunk
constexpr int kAqTile = kWave * kAqC;     // pixels per wave tile
constexpr int kAqRounds = 4;

// the group left open at a chunk end: min | max << 8 | 1 << 16, and its
// first pixel; mm == 0 is "no group" (the start of the sequence, or the
// speculative entry)
struct AqState {
    uint32_t mm;
    uint32_t pad;
    unsigned long long head;
};

struct AqCtl {
    uint32_t changed[kAqRounds + 1];
    uint32_t rounds;
    unsigned long long first_changed[kAqRounds + 1];
    unsigned long long finisher_chunks;
};

struct AqArgs {
    const uint8_t* D;
    uint8_t* Q;
    unsigned long long m;
    unsigned long long nchunks;
    uint32_t K;  // 2 * floor(E), at most 255 (255: one group)
    AqCtl* ctl;
    AqState* exitb;   // 2 * nchunks: the open group at each chunk end, by round parity
    AqState* used;    // nchunks: the entry each chunk's stored result was computed from
    AqState* spec;    // nchunks: the speculative chain's open group at the chunk end
    uint4* sheads;    // 2 * nchunks: the speculative chain's group starts, a bit per pixel
    uint16_t* closev; // nchunks: 0x100 | value of the entering group when it ends in the chunk, else 0
    uint8_t* gv;      // nchunks: value of the group that starts in chunk k and crosses its end
    unsigned long long* partial;  // per workgroup: groups counted by the write pass
    roix_absq_info* info;
};

__device__ __forceinline__ bool aq_same(const AqState& a, const AqState& b) {
    return a.mm == b.mm && a.head == b.head;
}

__device__ __forceinline__ uint32_t aq_pack(uint32_t mn, uint32_t mx) { return mn | (mx << 8) | 0x10000u; }
__device__ __forceinline__ uint32_t aq_mid(uint32_t mm) { return ((mm & 0xFFu) + ((mm >> 8) & 0xFFu)) >> 1; }

// Stage the wave's tile (chunks 64 t .. 64 t + 63) into LDS.
__device__ __forceinline__ void aq_load_tile(const AqArgs& a, unsigned long long t, uint32_t* lds, int lane) {
    const unsigned long long tile0 = t * (unsigned long long)kAqTile;
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two batches of 8 loads in flight
        uint4 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const unsigned long long g = tile0 + 16ull * lane + 1024ull * (8 * h + i);
            if (g + 16 <= a.m) {
                v[i] = ld_stream(reinterpret_cast<const uint4*>(a.D + g));
            } else {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
                for (int b = 0; b < 16; ++b)
                    if (g + b < a.m) w[b >> 2] |= (uint32_t)a.D[g + b] << (8 * (b & 3));
                v[i] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int o = 16 * lane + 1024 * (8 * h + i);
            uint32_t* p = lds + (o >> 8) * kAqStride + ((o & 255) >> 2);
            p[0] = v[i].x;
            p[1] = v[i].y;
            p[2] = v[i].z;
            p[3] = v[i].w;
        }
    }
}

__device__ __forceinline__ void aq_store_tile(const AqArgs& a, unsigned long long t, const uint32_t* lds, int lane) {
    const unsigned long long tile0 = t * (unsigned long long)kAqTile;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        const int o = 16 * lane + 1024 * i;
        const uint32_t* p = lds + (o >> 8) * kAqStride + ((o & 255) >> 2);
        const uint4 v = make_uint4(p[0], p[1], p[2], p[3]);
        const unsigned long long g = tile0 + (unsigned long long)o;
        if (g + 16 <= a.m) {
            *reinterpret_cast<uint4*>(a.Q + g) = v;
        } else {
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            for (int b = 0; b < 16; ++b)
                if (g + b < a.m) a.Q[g + b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
        }
    }
}

__device__ __forceinline__ int aq_len(const AqArgs& a, unsigned long long k) {
    if (k >= a.nchunks) return 0;
    const unsigned long long left = a.m - k * (unsigned long long)kAqC;
    return left < (unsigned long long)kAqC ? (int)left : kAqC;
}

// One pixel of the scan: the group (mn, mx) takes v, or v starts a group
// (max - min over the group would exceed K).  An empty group is
// mn = 255, mx = 0, and force starts a group whatever the values.
#define AQ_STEP(v, force)                                         \
    const uint32_t nmn = (v) < mn ? (v) : mn;                     \
    const uint32_t nmx = (v) > mx ? (v) : mx;                     \
    const bool head = (force) || nmx - nmn > K;                   \
    const uint32_t pmm = aq_pack(mn, mx);                         \
    mn = head ? (v) : nmn;                                        \
    mx = head ? (v) : nmx;                                        \
    (void)pmm;

// Rescan chunk k from the open group `entry` (never "no group": chunk 0 is
// never rescanned) until a group starts where one of the speculative chain
// starts: from there the two chains are the same.  Returns the open group at
// the chunk end and, in closev, the value of the entering group when it ends
// inside the chunk.
__device__ __forceinline__ AqState aq_rescan(const AqArgs& a, const uint32_t* row, unsigned long long k,
                                             const AqState& entry, uint32_t& closev) {
    const uint32_t K = a.K;
    const int len = aq_len(a, k);
    const uint32_t* sh = reinterpret_cast<const uint32_t*>(a.sheads + 2 * k);
    uint32_t mn = entry.mm & 0xFFu, mx = (entry.mm >> 8) & 0xFFu;
    int lh = -1;
    bool merged = false;
    uint32_t close = 0u;
#pragma unroll 1
    for (int seg = 0; seg < kAqC / 32 && seg * 32 < len; ++seg) {
        const uint32_t shw = sh[seg];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const uint32_t word = row[seg * 8 + w];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int jl = 4 * w + b;
                const int j = seg * 32 + jl;
                if (j < len) {
                    const uint32_t v = (word >> (8 * b)) & 0xFFu;
                    AQ_STEP(v, false)
                    close = (head && close == 0u) ? (0x100u | aq_mid(pmm)) : close;
                    lh = head ? j : lh;
                    merged = merged || (head && ((shw >> jl) & 1u));
                }
            }
            if (merged) break;
        }
        if (merged) break;
    }
    closev = close;
    if (merged) return a.spec[k];
    AqState ex;
    ex.mm = aq_pack(mn, mx);
    ex.pad = 0u;
    ex.head = lh >= 0 ? k * (unsigned long long)kAqC + (unsigned long long)lh : entry.head;
    return ex;
}

__global__ void k_aq_init(AqArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int r = 0; r <= kAqRounds; ++r) {
        a.ctl->changed[r] = 0u;
        a.ctl->first_changed[r] = ~0ull;
    }
    a.ctl->rounds = 0u;
    a.ctl->finisher_chunks = 0ull;
}

// Speculation: every chunk from a group starting at its first pixel.  The
// speculative chain's values are written as the output: every group after
// the point where the true chain meets this one is a true group already, so
// the last pass only repairs the part before that point and the group that
// crosses the chunk end.  The running value of the open group is kept at its
// first byte in LDS after every pixel, and a second sweep spreads them.
__global__ __launch_bounds__(kWave) void k_aq_spec(AqArgs a) {
    __shared__ uint32_t lds[kWave * kAqStride];
    __shared__ uint32_t hbs[kWave * 9];  // group starts of each lane's chunk, a bit per pixel
    const int lane = threadIdx.x;
    const uint32_t K = a.K;
    const unsigned long long ntiles = (a.nchunks + kWave - 1) / kWave;
    for (unsigned long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const unsigned long long k = t * kWave + (unsigned long long)lane;
        __syncthreads();
        aq_load_tile(a, t, lds, lane);
        __syncthreads();
        if (k < a.nchunks) {
            uint32_t* row = lds + lane * kAqStride;
            uint32_t* hb = hbs + lane * 9;
            uint8_t* bytes = reinterpret_cast<uint8_t*>(row);
            const int len = aq_len(a, k);
            uint32_t mn = 255u, mx = 0u;
            uint32_t* sh = reinterpret_cast<uint32_t*>(a.sheads + 2 * k);
            int lh = 0;
#pragma unroll 1
            for (int seg = 0; seg < kAqC / 32; ++seg) {
                uint32_t hbw = 0u;
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const uint32_t word = row[seg * 8 + w];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int jl = 4 * w + b;
                        const int j = seg * 32 + jl;
                        if (j < len) {
                            const uint32_t v = (word >> (8 * b)) & 0xFFu;
                            AQ_STEP(v, j == 0)
                            lh = head ? j : lh;
                            hbw |= head ? (1u << jl) : 0u;
                            bytes[lh] = (uint8_t)((mn + mx) >> 1);
                        }
                    }
                }
                sh[seg] = hbw;
                hb[seg] = hbw;
            }
            AqState ex;
            ex.mm = aq_pack(mn, mx);
            ex.pad = 0u;
            ex.head = k * (unsigned long long)kAqC + (unsigned long long)lh;
            a.spec[k] = ex;
            a.exitb[k] = ex;  // round parity 0
            a.used[k] = AqState{0u, 0u, 0ull};
            a.closev[k] = 0;
            // spread each group's value from its first byte
            uint32_t cur = 0u;
#pragma unroll 1
            for (int seg = 0; seg < kAqC / 32; ++seg) {
                const uint32_t hbw = hb[seg];
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const uint32_t word = row[seg * 8 + w];
                    uint32_t o = 0u;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if ((hbw >> (4 * w + b)) & 1u) cur = (word >> (8 * b)) & 0xFFu;
                        o |= cur << (8 * b);
                    }
                    row[seg * 8 + w] = o;
                }
            }
        }
        __syncthreads();
        aq_store_tile(a, t, lds, lane);
    }
}

// Round r >= 1: every chunk whose entry (its predecessor's open group in
// round r - 1) differs from the one its stored result came from is rescanned.
__global__ __launch_bounds__(kWave) void k_aq_round(AqArgs a, int r) {
    __shared__ uint32_t lds[kWave * kAqStride];
    if (r >= 2 && __hip_atomic_load(&a.ctl->changed[r - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        return;  // the previous round changed nothing: every chunk is settled
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0) a.ctl->rounds = (uint32_t)r;
    const AqState* prev = a.exitb + (size_t)((r + 1) & 1) * a.nchunks;
    AqState* cur = a.exitb + (size_t)(r & 1) * a.nchunks;
    const unsigned long long ntiles = (a.nchunks + kWave - 1) / kWave;
    bool changed = false;
    unsigned long long first = ~0ull;
    for (unsigned long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const unsigned long long k = t * kWave + (unsigned long long)lane;
        const bool live = k < a.nchunks;
        AqState entry = {0u, 0u, 0ull};
        bool need = false;
        if (live && k >= 1) {
            entry = prev[k - 1];
            need = !aq_same(entry, a.used[k]);
        }
        if (__ballot(need) != 0ull) {
            __syncthreads();  // the previous tile's LDS reads are done
            aq_load_tile(a, t, lds, lane);
            __syncthreads();
        }
        if (need) {
            uint32_t cv;
            const AqState ex = aq_rescan(a, lds + lane * kAqStride, k, entry, cv);
            a.used[k] = entry;
            a.closev[k] = (uint16_t)cv;
            cur[k] = ex;
            if (!aq_same(ex, prev[k])) {
                changed = true;
                first = k < first ? k : first;
            }
        } else if (live) {
            cur[k] = prev[k];
        }
    }
    first = wave_min(first);
    if (__ballot(changed) != 0ull && lane == 0) {
        a.ctl->changed[r] = 1u;
        atomicMin(&a.ctl->first_changed[r], first);
    }
}

// Settle, in order, the chunks the rounds left inconsistent (an entry that is
// not the predecessor's final open group).  One wave; checks 64 chunks per
// step and rescans the first inconsistent one on lane 0.  Every step moves
// the cursor forward, so the loop ends.
__global__ __launch_bounds__(kWave) void k_aq_finish(AqArgs a) {
    __shared__ uint32_t row[kAqStride];
    if (__hip_atomic_load(&a.ctl->changed[kAqRounds], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    const int lane = threadIdx.x;
    AqState* ex = a.exitb + (size_t)(kAqRounds & 1) * a.nchunks;
    unsigned long long k = a.ctl->first_changed[kAqRounds] + 1;
    bool fresh = false;  // lane 0's register holds the exit of chunk k - 1 just rescanned
    AqState last = {0u, 0u, 0ull};
    unsigned long long done = 0;
    while (k < a.nchunks) {
        const unsigned long long kk = k + (unsigned long long)lane;
        bool bad = false;
        AqState in = {0u, 0u, 0ull};
        if (kk < a.nchunks) {
            in = (lane == 0 && fresh) ? last : ex[kk - 1];
            bad = !aq_same(in, a.used[kk]);
        }
        const unsigned long long mask = __ballot(bad);
        if (mask == 0ull) {
            k += kWave;
            fresh = false;
            continue;
        }
        const int f = __ffsll((unsigned long long)mask) - 1;
        const unsigned long long c = k + (unsigned long long)f;
        AqState entry;
        entry.mm = __shfl(in.mm, f);
        entry.pad = 0u;
        entry.head = __shfl(in.head, f);
        __syncthreads();
        {  // chunk c into LDS: 4 bytes per lane
            const unsigned long long g = c * (unsigned long long)kAqC + 4ull * lane;
            uint32_t w = 0u;
            for (int b = 0; b < 4; ++b)
                if (g + b < a.m) w |= (uint32_t)a.D[g + b] << (8 * b);
            row[lane] = w;
        }
        __syncthreads();
        if (lane == 0) {
            uint32_t cv;
            last = aq_rescan(a, row, c, entry, cv);
            ex[c] = last;
            a.used[c] = entry;
            a.closev[c] = (uint16_t)cv;
        }
        ++done;
        fresh = true;
        k = c + 1;
    }
    if (lane == 0) a.ctl->finisher_chunks = done;
}

// The value of each group that crosses a chunk end, from the chunk where it
// ends (or from the end of the sequence), into slot gv[chunk of its head].
__global__ __launch_bounds__(256) void k_aq_close(AqArgs a) {
    const AqState* ex = a.exitb + (size_t)(kAqRounds & 1) * a.nchunks;
    const unsigned long long n = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; k < a.nchunks; k += n) {
        if (k >= 1) {
            const uint32_t cv = a.closev[k];
            if (cv & 0x100u) a.gv[ex[k - 1].head / kAqC] = (uint8_t)(cv & 0xFFu);
        }
        if (k == a.nchunks - 1) {
            const AqState e = ex[k];
            a.gv[e.head / kAqC] = (uint8_t)aq_mid(e.mm);
        }
    }
}

// The output's repair: each chunk is rescanned from its settled entry (its
// predecessor's final open group) until a group starts where a speculative
// one does; the bytes before that point are rewritten with the true groups'
// values (the entering group's from its slot), and the group open at the
// chunk end gets its value from its slot.  A chunk whose true chain never
// meets the speculative one is rewritten whole.  Counts the true groups.
// Pixels are read 16 at a time from global memory, as far as the rescan
// goes; bytes are written one by one.
__device__ __forceinline__ void aq_fill(uint8_t* q, int from, int to, uint32_t v) {
    for (int j = from; j < to; ++j) q[j] = (uint8_t)v;
}

__global__ __launch_bounds__(256) void k_aq_fix(AqArgs a) {
    const uint32_t K = a.K;
    const AqState* ex = a.exitb + (size_t)(kAqRounds & 1) * a.nchunks;
    unsigned long long groups = 0;
    const unsigned long long n = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; k < a.nchunks; k += n) {
        const int len = aq_len(a, k);
        const uint32_t* sh = reinterpret_cast<const uint32_t*>(a.sheads + 2 * k);
        const AqState spec = a.spec[k];
        const int spec_last = (int)(spec.head - k * (unsigned long long)kAqC);
        uint8_t* q = a.Q + k * (unsigned long long)kAqC;
        if (k == 0) {  // the sequence starts here: the true chain is the speculative one
            int c = 0;
            for (int i = 0; i < kAqC / 32; ++i) c += __popc(sh[i]);
            groups += (unsigned long long)c;
            if (a.nchunks > 1) aq_fill(q, spec_last, len, a.gv[0]);
            continue;
        }
        const AqState entry = ex[k - 1];
        const uint32_t lead = a.gv[entry.head / kAqC];
        uint32_t mn = entry.mm & 0xFFu, mx = (entry.mm >> 8) & 0xFFu;
        int s = -1;  // first pixel of the true group being scanned (-1: the entering group)
        int p = -1;  // where the chains meet
        int own = 0;  // true group starts before p
        const uint4* d = reinterpret_cast<const uint4*>(a.D + k * (unsigned long long)kAqC);
        uint4 blk = make_uint4(0u, 0u, 0u, 0u);
        for (int j = 0; j < len && p < 0; ++j) {
            if ((j & 15) == 0) {  // the next 16 pixels (whole within the buffer, or the last chunk's tail)
                if (k * (unsigned long long)kAqC + (unsigned long long)j + 16ull <= a.m) {
                    blk = d[j >> 4];
                } else {
                    uint32_t w[4] = {0u, 0u, 0u, 0u};
                    for (int b = 0; b < 16 && j + b < len; ++b)
                        w[b >> 2] |= (uint32_t)a.D[k * (unsigned long long)kAqC + j + b] << (8 * (b & 3));
                    blk = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
            const uint32_t wd = (j & 8) ? ((j & 4) ? blk.w : blk.z) : ((j & 4) ? blk.y : blk.x);
            const uint32_t v = (wd >> (8 * (j & 3))) & 0xFFu;
            const uint32_t nmn = v < mn ? v : mn, nmx = v > mx ? v : mx;
            if (nmx - nmn > K) {  // a true group starts at j
                if (s < 0) aq_fill(q, 0, j, lead);
                else aq_fill(q, s, j, (mn + mx) >> 1);
                if ((sh[j >> 5] >> (j & 31)) & 1u) {
                    p = j;
                    break;
                }
                ++own;
                s = j;
                mn = mx = v;
            } else {
                mn = nmn;
                mx = nmx;
            }
        }
        if (p >= 0) {  // from p on the speculative chain's values stand, but for the group crossing the end
            int c = own;
            for (int i = 0; i < kAqC / 32; ++i) {
                const uint32_t w = sh[i];
                const int lo = i * 32;
                const uint32_t m = p <= lo ? ~0u : (p >= lo + 32 ? 0u : (~0u << (p - lo)));
                c += __popc(w & m);
            }
            groups += (unsigned long long)c;
            if (k + 1 < a.nchunks) aq_fill(q, spec_last, len, a.gv[k]);
            // the last chunk's final group ends with the sequence: its value is the speculation's
        } else {  // never met: the true groups throughout
            groups += (unsigned long long)own;
            const uint32_t tv = s < 0 ? lead : (k + 1 < a.nchunks ? a.gv[k] : ((mn + mx) >> 1));
            aq_fill(q, s < 0 ? 0 : s, len, tv);
        }
    }
    groups = wave_sum(groups);
    __shared__ unsigned long long part[256 / kWave];
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = groups;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int i = 0; i < 256 / kWave; ++i) sum += part[i];
        a.partial[blockIdx.x] = sum;
    }
}

__global__ __launch_bounds__(256) void k_aq_finalize(AqArgs a, int nparts, int32_t status) {
    __shared__ unsigned long long s[256];
    unsigned long long v = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) v += a.partial[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.info->status = status;
        a.info->rounds = (int32_t)a.ctl->rounds;
        a.info->n_groups = s[0];
        a.info->finisher_chunks = a.ctl->finisher_chunks;
        a.info->pad = 0ull;
    }
}

constexpr int kAqMaxGrid = 8192;  // workgroups (one wave each) of the tile passes

static size_t aq_align(size_t x) { return (x + 255) & ~(size_t)255; }

size_t absq_scratch_bytes(int64_t m) {
    const size_t nchunks = (size_t)((m + kAqC - 1) / kAqC);
    return aq_align(sizeof(AqCtl)) + aq_align(nchunks * sizeof(AqState) * 4) + aq_align(nchunks * 32) +
           aq_align(nchunks * 2) + aq_align(nchunks) + aq_align((size_t)kAqMaxGrid * 8);
}

static int absq_grid(const LaunchCtx& lc, int64_t m) {
    const int64_t ntiles = (m + kAqTile - 1) / kAqTile;
    int64_t cap = (int64_t)lc.grid_stream * 4;
    cap = cap < kAqMaxGrid ? cap : kAqMaxGrid;
    return (int)(ntiles < 1 ? 1 : ntiles < cap ? ntiles : cap);
}

hipError_t launch_absq(const LaunchCtx& lc, const uint8_t* D, int64_t m, uint32_t K, uint8_t* Q, void* scratch,
                       roix_absq_info* info) {
    static_assert(kAqTile == 16 * 1024, "a wave tile is 16 loads of 16 bytes per lane");
    const int grid = absq_grid(lc, m);
    uint8_t* p = (uint8_t*)scratch;
    AqArgs a;
    a.D = D;
    a.Q = Q;
    a.m = (unsigned long long)m;
    a.nchunks = (unsigned long long)((m + kAqC - 1) / kAqC);
    a.K = K;
    a.ctl = (AqCtl*)p;
    p += aq_align(sizeof(AqCtl));
    a.exitb = (AqState*)p;
    a.used = a.exitb + 2 * a.nchunks;
    a.spec = a.used + a.nchunks;
    p += aq_align((size_t)a.nchunks * sizeof(AqState) * 4);
    a.sheads = (uint4*)p;
    p += aq_align((size_t)a.nchunks * 32);
    a.closev = (uint16_t*)p;
    p += aq_align((size_t)a.nchunks * 2);
    a.gv = p;
    p += aq_align((size_t)a.nchunks);
    a.partial = (unsigned long long*)p;
    a.info = info;
    timer_begin(lc.timer, ST_ABSQ, lc.stream);
    // chunk-per-thread kernels (close, repair): at most kAqMaxGrid partial counts
    const int cgrid = (int)((a.nchunks + 255) / 256 < 4096 ? (a.nchunks + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_aq_init, dim3(1), dim3(64), 0, lc.stream, a);
    if (m > 0) {
        hipLaunchKernelGGL(k_aq_spec, dim3(grid), dim3(kWave), 0, lc.stream, a);
        for (int r = 1; r <= kAqRounds; ++r)
            hipLaunchKernelGGL(k_aq_round, dim3(grid), dim3(kWave), 0, lc.stream, a, r);
        hipLaunchKernelGGL(k_aq_finish, dim3(1), dim3(kWave), 0, lc.stream, a);
        hipLaunchKernelGGL(k_aq_close, dim3(cgrid), dim3(256), 0, lc.stream, a);
        hipLaunchKernelGGL(k_aq_fix, dim3(cgrid), dim3(256), 0, lc.stream, a);
    }
    hipLaunchKernelGGL(k_aq_finalize, dim3(1), dim3(256), 0, lc.stream, a, m > 0 ? cgrid : 0, 0);
    timer_end(lc.timer, ST_ABSQ, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
