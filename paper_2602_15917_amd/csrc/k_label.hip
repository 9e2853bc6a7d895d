// k_label.hip - binary mask, foreground runs, 3-D connected components of the
// runs, per-component statistics and the keep rule.
//
// The mask (object = proxy byte above the threshold byte) is turned into a
// row bitmask with SWAR byte compares, and every row (z, y) into its maximal
// runs of object voxels.  Runs are numbered in raster order, so the run with
// the smallest number of a component holds the component's smallest linear
// voxel index.  Touching runs of neighbouring rows are united with a union-
// find that always links the larger root under the smaller one: first in
// LDS within segments of consecutive run numbers, then across segments in
// the global forest.  After flattening, the root of a component is its first
// run and the canonical label is that run's first voxel.  Work is O(runs),
// not O(voxels): per-voxel traffic is one read of the 1-byte proxy and one
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

// Workgroups of a pass over the runs (or components) of a volume of nrows
// rows, planned for kPlanRuns runs a row: the run count is device data, and
// the passes stride over any count, so the grid only sets their speed; a
// small volume (or each small volume of a batch) then launches few
// workgroups, a large one the cap.
constexpr int kPlanRuns = 8;
static int runs_grid(int64_t nrows, int runs_per_block, int cap) {
    return grid_for(nrows * kPlanRuns, runs_per_block, cap);
}

// ------------------------------------------------------- mask bits + counts

// Bytes of v above the threshold t, as 4 bits: with T = 255 - t, byte b > t
// exactly when b + T carries out of 8 bits.  The carry into bit 7 is bit 7 of
// the 7-bit partial sums (no carry crosses a byte), the carry out of bit 7 is
// the full-adder majority; a multiply gathers the four carry bits.
__device__ __forceinline__ uint32_t gt_bytes4(uint32_t v, uint32_t TL, uint32_t TR) {
    const uint32_t lo = (v & 0x7F7F7F7Fu) + TL;
    const uint32_t c = ((v & TR) | (lo & (v | TR))) & 0x80808080u;
    return (((c >> 7) * 0x00204081u) >> 21) & 0xFu;
}

// mask word of 64 proxy bytes (four 16-byte loads)
__device__ __forceinline__ uint64_t mask_word(const uint8_t* p, uint32_t TL, uint32_t TR) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    const uint4 a = q[0], b = q[1], c = q[2], d = q[3];
    const uint32_t dw[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) lo |= gt_bytes4(dw[i], TL, TR) << (4 * i);
#pragma unroll
    for (int i = 0; i < 8; ++i) hi |= gt_bytes4(dw[8 + i], TL, TR) << (4 * i);
    return ((uint64_t)hi << 32) | lo;
}

// The 64 mask words of proxy words [wbase, wbase + 64) (valid: the first
// nvalid of them), lane l returning word l.  The bytes are loaded coalesced --
// lane l takes bytes 16 l .. 16 l + 15 of each 1 KB -- and turned into 16 mask
// bits each; word w then gathers its four quarters from lanes 4 (w % 16) + q
// of load w / 16.  Every lane of the wave must call it.
__device__ __forceinline__ void mask_load64(const uint8_t* proxy, int64_t wbase, int64_t nvalid, uint4 (&v)[4]) {
    const int lane = threadIdx.x % kWave;
    const uint4* src = reinterpret_cast<const uint4*>(proxy + wbase * 64) + lane;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = k * 16 + lane / 4 < nvalid ? ld_stream(src + k * 64) : make_uint4(0, 0, 0, 0);
}

// zero bytes are never above the threshold, so the loads' zero fill is empty mask
__device__ __forceinline__ uint64_t mask_words64(const uint4 (&v)[4], const uint32_t (&TL)[4],
                                                 const uint32_t (&TR)[4]) {
    const int lane = threadIdx.x % kWave;
    uint32_t h[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        h[k] = gt_bytes4(v[k].x, TL[k], TR[k]) | (gt_bytes4(v[k].y, TL[k], TR[k]) << 4) |
               (gt_bytes4(v[k].z, TL[k], TR[k]) << 8) | (gt_bytes4(v[k].w, TL[k], TR[k]) << 12);
    const uint32_t h01 = h[0] | (h[1] << 16), h23 = h[2] | (h[3] << 16);
    const int k = lane >> 4, m4 = (lane & 15) * 4;
    uint64_t word = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t a = (uint32_t)__shfl((int)h01, m4 + q), b = (uint32_t)__shfl((int)h23, m4 + q);
        const uint32_t srcv = k < 2 ? a : b;
        const uint32_t bits = (k & 1) ? (srcv >> 16) : (srcv & 0xFFFFu);
        word |= (uint64_t)bits << (16 * q);
    }
    return word;
}

// 16-bit proxy (low 15 bits of q, outlier flag in bit 15), two voxels per
// dword, with 16-bit lane adds (no carry between the halves): the low 15 bits
// of p + 2^15 - qmin15 are q - qmin, and bit 15 of that plus 2^15 - tq is set
// exactly when q - qmin >= tq (q - qmin < 2^15, 0 <= tq <= 2^15).  Returns
// the 8 mask bits of 8 voxels (voxel i at bit i).
typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t add_u16x2(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2_t, a) + __builtin_bit_cast(u16x2_t, b));
}
__device__ __forceinline__ uint32_t ge_halves8(const uint4& v, uint32_t A2, uint32_t T2) {
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
    uint32_t z[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = add_u16x2(add_u16x2(d[i], A2) & 0x7FFF7FFFu, T2) & 0x80008000u;
    // bit 15 of dword i to bit 2 i, bit 31 to bit 2 i + 16, then fold
    const uint32_t y = (z[0] >> 15) | (z[1] >> 13) | (z[2] >> 11) | (z[3] >> 9);
    return (y & 0x55u) | ((y >> 15) & 0xAAu);
}

// mask word of 64 16-bit proxy elements (eight 16-byte loads)
__device__ __forceinline__ uint64_t mask_word16(const uint16_t* p, uint32_t Q2, uint32_t T2) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q[k];
    uint64_t m = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) m |= (uint64_t)ge_halves8(v[k], Q2, T2) << (8 * k);
    return m;
}

// As mask_load64 for the 16-bit proxy: lane l takes bytes 16 l .. 16 l + 15
// of each 1 KB, eight loads for 64 words; word w gathers its eight 8-bit
// pieces from lanes 8 (w % 8) + j of load w / 8.  Invalid words load zeros,
// which the caller clears.
__device__ __forceinline__ void mask_load64_16(const uint16_t* proxy, int64_t wbase, int64_t nvalid,
                                               uint4 (&v)[8]) {
    const int lane = threadIdx.x % kWave;
    const uint4* src = reinterpret_cast<const uint4*>(proxy + wbase * 64) + lane;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = k * 8 + lane / 8 < nvalid ? ld_stream(src + k * 64) : make_uint4(0, 0, 0, 0);
}

// Word assembly for mask_load64_16's layout.  Lane 8 g + j holds in byte k
// of (hi:lo) the 8 mask bits of bits 8 j .. 8 j + 7 of word 8 k + g.  An
// 8 x 8 byte transpose inside each group of 8 lanes (three butterfly stages
// by DPP: at lane distance 4, 2, 1 a lane sends the four bytes it replaces
// and takes its partner's) leaves word 8 k + g whole in lane 8 g + k; one
// lane permutation then hands word l to lane l.
__device__ __forceinline__ uint64_t words_from_bytes8(uint32_t lo, uint32_t hi) {
    const int lane = threadIdx.x % kWave;
    {  // distance 4: the low lanes send bytes 4-7, the high ones bytes 0-3
        const bool up = lane & 4;
        const uint32_t snd = up ? lo : hi;
        const uint32_t from_above = dpp_u32<kDppRowShl + 4>(0u, snd), from_below = dpp_u32<kDppRowShr + 4>(0u, snd);
        if (up)
            lo = from_below;
        else
            hi = from_above;
    }
    {  // distance 2: bytes 2, 3, 6, 7 of the lanes with bit 1 clear, 0, 1, 4, 5 of the others
        const bool up = lane & 2;
        const uint32_t snd = __builtin_amdgcn_perm(hi, lo, up ? 0x05040100u : 0x07060302u);
        const uint32_t got = dpp_u32<kDppQuadXor2>(0u, snd);
        lo = __builtin_amdgcn_perm(got, lo, up ? 0x03020504u : 0x05040100u);
        hi = __builtin_amdgcn_perm(got, hi, up ? 0x03020706u : 0x07060100u);
    }
    {  // distance 1: odd bytes of the even lanes, even bytes of the odd ones
        const bool up = lane & 1;
        const uint32_t snd = __builtin_amdgcn_perm(hi, lo, up ? 0x06040200u : 0x07050301u);
        const uint32_t got = dpp_u32<kDppQuadXor1>(0u, snd);
        lo = __builtin_amdgcn_perm(got, lo, up ? 0x03050104u : 0x05020400u);
        hi = __builtin_amdgcn_perm(got, hi, up ? 0x03070106u : 0x07020600u);
    }
    const int src = 8 * (lane & 7) + (lane >> 3);
    const uint32_t wlo = (uint32_t)__shfl((int)lo, src), whi = (uint32_t)__shfl((int)hi, src);
    return (uint64_t)wlo | ((uint64_t)whi << 32);
}

__device__ __forceinline__ uint64_t mask_words64_16(const uint4 (&v)[8], uint32_t Q2, uint32_t T2) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) lo |= ge_halves8(v[k], Q2, T2) << (8 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k) hi |= ge_halves8(v[4 + k], Q2, T2) << (8 * k);
    return words_from_bytes8(lo, hi);
}

// uint16 volumes read directly: a voxel is object when its code reaches the
// threshold code, q(x) >= q_thr.  q(x) = rint(x r) never decreases with x,
// so that holds exactly for x >= X, the smallest such value (65536: none).
__device__ __forceinline__ uint32_t u16_threshold(float r, int32_t q_thr) {
    if (qcode(65535.0f, r) < q_thr) return 65536u;
    uint32_t lo = 0u, hi = 65535u;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (qcode((float)mid, r) >= q_thr)
            hi = mid;
        else
            lo = mid + 1u;
    }
    return lo;
}

// 8 mask bits of 8 uint16 values >= X (X2 = X in both halves, X <= 65535):
// the saturating difference X - x is zero exactly then, and bit 15 of
// (d & 0x7FFF) + 0x7FFF, or of d, is set exactly when a half d is not zero.
__device__ __forceinline__ uint32_t ge_u16x8(const uint4& v, uint32_t X2) {
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
    uint32_t z[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t r = __builtin_bit_cast(
            uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2_t, X2), __builtin_bit_cast(u16x2_t, d[i])));
        z[i] = ~(add_u16x2(r & 0x7FFF7FFFu, 0x7FFF7FFFu) | r) & 0x80008000u;
    }
    const uint32_t y = (z[0] >> 15) | (z[1] >> 13) | (z[2] >> 11) | (z[3] >> 9);
    return (y & 0x55u) | ((y >> 15) & 0xAAu);
}

// the mask words of mask_load64_16's loads, for uint16 values (all 0 when X2 is 0xFFFFFFFF)
__device__ __forceinline__ uint64_t mask_words64_u16(const uint4 (&v)[8], uint32_t X2, bool none) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) lo |= ge_u16x8(v[k], X2) << (8 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k) hi |= ge_u16x8(v[4 + k], X2) << (8 * k);
    if (none) lo = hi = 0u;
    return words_from_bytes8(lo, hi);
}

// Lane-per-word mapping of a wave step: with W <= 64 words per row, a step
// covers R = 64 / W rows, lane l holding word l % W of row l / W.
struct WordLane {
    int64_t row;   // -1 for an idle lane
    int64_t w;     // word index in the row
    int seg_first; // first lane of this lane's row in the wave
};

__device__ __forceinline__ WordLane word_lane(int64_t row0, int64_t W, int64_t nrows) {
    const int lane = threadIdx.x % kWave;
    const int R = (int)(kWave / W);
    const int rr = lane / (int)W;
    WordLane wl;
    wl.w = lane - rr * (int)W;
    wl.seg_first = rr * (int)W;
    wl.row = (rr < R && row0 + rr < nrows) ? row0 + rr : -1;
    return wl;
}

// SWAR constants of "byte > t" for the slice of row `row` (per-slice
// thresholds thr[z]; z0 = the slice of a row at or before `row`).
__device__ __forceinline__ void slice_consts(const int32_t* __restrict__ thr, int64_t row, int64_t z0, int64_t ny,
                                             uint32_t& TL, uint32_t& TR) {
    int64_t z = z0;
    while (row >= (z + 1) * ny) ++z;
    const uint32_t T = 255u - (uint32_t)thr[z];
    TR = T * 0x01010101u;
    TL = (T & 0x7Fu) * 0x01010101u;
}

// One 64-bit mask word per lane (SWAR byte compares on 64 proxy bytes), run
// starts = 1-bits whose left neighbour (previous bit, or the previous lane's
// top bit) is 0, per-row run counts by a segmented wave scan.  slice_thr
// (1-byte proxy only): a threshold bin per z-slice instead of one.  MODE 0:
// 1-byte bin proxy; 1: 16-bit code proxy; 2: the uint16 volume itself, rows
// of whole 64-voxel words (its rows are then laid out as the 16-bit proxy's).
template <int MODE, bool NT>
__device__ __forceinline__ void mask_runs_body(const VPart vp, const uint8_t* __restrict__ proxy, int64_t nx,
                                               int64_t nrows, int64_t W,
                                               DevState* S, uint64_t* __restrict__ maskbits,
                                               uint32_t* __restrict__ row_nruns, const int32_t* __restrict__ slice_thr,
                                               int64_t ny) {
    // 1-byte proxy: bin > threshold bin, by SWAR byte compares
    const uint32_t T = 255u - (uint32_t)S->proxy_thr;
    const uint32_t TR = T * 0x01010101u, TL = (T & 0x7Fu) * 0x01010101u;
    // 16-bit proxy: q - qmin >= q_thr - qmin
    const uint32_t Q2 = (0x8000u - ((uint32_t)S->qmin & 0x7FFFu)) * 0x00010001u;
    const uint32_t T2 = (0x8000u - (uint32_t)((int64_t)S->q_thr - (int64_t)S->qmin)) * 0x00010001u;
    constexpr bool P16 = MODE != 0;
    uint32_t X2 = 0u;
    bool none = false;
    if constexpr (MODE == 2) {
        const uint32_t X = u16_threshold(S->r, S->q_thr);
        none = X > 65535u;
        X2 = (none ? 65535u : X) * 0x00010001u;
    }
    const uint16_t* proxy16 = reinterpret_cast<const uint16_t*>(proxy);
    const uint64_t lastmask = (nx % 64) ? ((1ull << (nx % 64)) - 1ull) : ~0ull;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)vp.b * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)vp.n * blockDim.x / kWave;
    const int64_t P = W * 64;
    unsigned long long nmask = 0;
    if (W <= kWave) {
        const int64_t R = kWave / W;
        // rows of the step at row0 (its rows are consecutive words of the
        // proxy: lane l's word is word l)
        auto rows_at = [&](int64_t row0) -> int64_t { return row0 >= nrows ? 0 : (nrows - row0 < R ? nrows - row0 : R); };
        auto finish = [&](uint64_t m, int64_t row0) {
            const WordLane wl = word_lane(row0, W, nrows);
            if (wl.row < 0)
                m = 0;
            else if (wl.w == W - 1)
                m &= lastmask;
            const uint32_t prev_hi = dpp_u32<kDppWaveShr1>(0u, (uint32_t)(m >> 32));
            const uint64_t cin = (wl.w > 0) ? (uint64_t)(prev_hi >> 31) : 0ull;
            const uint64_t starts = m & ~((m << 1) | cin);
            const uint32_t cnt = (uint32_t)__popcll(starts);
            nmask += (unsigned long long)__popcll(m);
            const uint32_t incl = wave_incl_scan(cnt);
            const uint32_t before = __shfl(incl, wl.seg_first > 0 ? wl.seg_first - 1 : 0);
            if (wl.row >= 0) {
                if constexpr (NT)
                    __builtin_nontemporal_store((unsigned long long)m,
                                                reinterpret_cast<unsigned long long*>(maskbits + wl.row * W + wl.w));
                else
                    maskbits[wl.row * W + wl.w] = m;
                if (wl.w == W - 1) row_nruns[wl.row] = incl - (wl.seg_first > 0 ? before : 0u);
            }
        };
        if constexpr (P16) {
            auto words = [&](const uint4 (&v)[8]) {
                if constexpr (MODE == 2)
                    return mask_words64_u16(v, X2, none);
                else
                    return mask_words64_16(v, Q2, T2);
            };
            int64_t s = wave;  // step s covers rows s R .. s R + R - 1
            if (R * W == kWave) {
                // Steps of exactly 64 words: every load unconditional, so the
                // next step's eight loads stay in flight while this step's
                // words are formed (two register sets taking turns).  With no
                // next whole step the wave loads the volume's first step in
                // its place (in L2, never used).
                const int64_t nfull = nrows / R;
                const uint4* vb = reinterpret_cast<const uint4*>(proxy16) + lane;
                auto load = [&](int64_t st, uint4 (&v)[8]) {
                    const uint4* p = st < nfull ? vb + st * (kWave * 8) : vb;
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = ld_stream(p + k * kWave);
                };
                uint4 a[8], b[8];
                if (s < nfull) {
                    load(s, a);
                    for (;;) {
                        load(s + nwaves, b);
                        finish(words(a), s * R);
                        s += nwaves;
                        if (s >= nfull) break;
                        load(s + nwaves, a);
                        finish(words(b), s * R);
                        s += nwaves;
                        if (s >= nfull) break;
                    }
                }
            }
            // other row widths, and a last step of fewer rows
            for (; s * R < nrows; s += nwaves) {
                uint4 v[8];
                mask_load64_16(proxy16, s * R * W, rows_at(s * R) * W, v);
                finish(words(v), s * R);
            }
        } else {
            // two steps per iteration, all loads of both issued first
            for (int64_t rowA = wave * 2 * R; rowA < nrows; rowA += nwaves * 2 * R) {
                uint4 v[2][4];
#pragma unroll
                for (int u = 0; u < 2; ++u) mask_load64(proxy, (rowA + u * R) * W, rows_at(rowA + u * R) * W, v[u]);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int64_t row0 = rowA + u * R;
                    uint32_t tl[4] = {TL, TL, TL, TL}, tr[4] = {TR, TR, TR, TR};
                    if (slice_thr) {  // uniform
                        // load k of this lane holds word 16 k + lane / 4 of the step
                        const int64_t r0 = row0 < nrows ? row0 : nrows - 1;
                        const int64_t z0 = r0 / ny;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int64_t rr = (16 * k + lane / 4) / W;
                            const int64_t rk = rr < R && row0 + rr < nrows ? row0 + rr : r0;
                            slice_consts(slice_thr, rk, z0, ny, tl[k], tr[k]);
                        }
                    }
                    finish(mask_words64(v[u], tl, tr), row0);
                }
            }
        }
    } else {
        // long rows: one row per wave, 64 words per step, carries between steps
        for (int64_t row = wave; row < nrows; row += nwaves) {
            uint32_t carry = 0, total = 0;
            uint32_t tl = TL, tr = TR;
            if (!P16 && slice_thr) slice_consts(slice_thr, row, row / ny, ny, tl, tr);
            for (int64_t w0 = 0; w0 < W; w0 += kWave) {
                const int64_t w = w0 + lane;
                uint64_t m = 0;
                if (w < W) {
                    if constexpr (MODE == 2) {
                        const uint4* q = reinterpret_cast<const uint4*>(proxy16 + row * P + 64 * w);
#pragma unroll
                        for (int k = 0; k < 8; ++k) m |= none ? 0ull : (uint64_t)ge_u16x8(q[k], X2) << (8 * k);
                    } else if constexpr (P16)
                        m = mask_word16(proxy16 + row * P + 64 * w, Q2, T2);
                    else
                        m = mask_word(proxy + row * P + 64 * w, tl, tr);
                    if (w == W - 1) m &= lastmask;
                }
                const uint32_t hi = (uint32_t)(m >> 32);
                const uint32_t prev_hi = __shfl_up(hi, 1);
                const uint64_t cin = lane > 0 ? (uint64_t)(prev_hi >> 31) : (uint64_t)carry;
                const uint64_t starts = m & ~((m << 1) | cin);
                total += wave_sum((uint32_t)__popcll(starts));
                nmask += (unsigned long long)__popcll(m);
                carry = __shfl(hi, kWave - 1) >> 31;
                if (w < W) maskbits[row * W + w] = m;
            }
            if (lane == 0) row_nruns[row] = total;
        }
    }
    nmask = wave_sum(nmask);
    __shared__ unsigned long long s_n[kBlock / kWave];
    if (lane == 0) s_n[threadIdx.x / kWave] = nmask;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t += s_n[k];
        if (t) atomicAdd(&S->n_mask, t);
    }
}

// The proxy's kind is device data (the fused pass decides it); the branch is
// uniform.  u16: `proxy` is the uint16 volume (host-known).
__device__ __forceinline__ void k_mask_runs_body(const VPart vp, const uint8_t* __restrict__ proxy, int64_t nx, int64_t nrows,
                                                      int64_t W, DevState* S, uint64_t* __restrict__ maskbits,
                                                      uint32_t* __restrict__ row_nruns,
                                                      const int32_t* __restrict__ slice_thr, int64_t ny, int u16,
                                                      int nt_words) {
    if (block_exit_l(S)) return;
    // NT: mask words stored non-temporally
    if (u16) {
        if (nt_words)
            mask_runs_body<2, true>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, nullptr, ny);
        else
            mask_runs_body<2, false>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, nullptr, ny);
    } else if (S->p16) {
        if (nt_words)
            mask_runs_body<1, true>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, nullptr, ny);
        else
            mask_runs_body<1, false>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, nullptr, ny);
    } else {
        if (nt_words)
            mask_runs_body<0, true>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, slice_thr, ny);
        else
            mask_runs_body<0, false>(vp, proxy, nx, nrows, W, S, maskbits, row_nruns, slice_thr, ny);
    }
}
__global__ __launch_bounds__(kBlock) void k_mask_runs(const uint8_t* __restrict__ proxy, int64_t nx, int64_t nrows,
                                                      int64_t W, DevState* S, uint64_t* __restrict__ maskbits,
                                                      uint32_t* __restrict__ row_nruns,
                                                      const int32_t* __restrict__ slice_thr, int64_t ny, int u16,
                                                      int nt_words) {
    k_mask_runs_body(hw_part(), proxy, nx, nrows, W, S, maskbits, row_nruns, slice_thr, ny, u16, nt_words);
}

hipError_t launch_mask_runs(const LaunchCtx& lc, const Geom& g, const Layout& L, const int32_t* slice_thr,
                            const uint16_t* u16_in) {
    timer_begin(lc.timer, ST_MASK_RUNS, lc.stream);
    const int64_t R = g.W <= kWave ? kWave / g.W : 1;
    int grid = grid_for((g.nrows + R - 1) / R, kBlock / kWave, lc.grid_mask);
    const uint8_t* src = u16_in ? reinterpret_cast<const uint8_t*>(u16_in) : (const uint8_t*)L.proxy;
    // Mask words that fit the last-level cache are stored normally: the run
    // pass reads them straight back.  Larger ones are streamed out, so they
    // do not evict the proxy lines still to be read.
    const int nt_words = g.nrows * g.W * (int64_t)sizeof(uint64_t) > kLastLevelCache ? 1 : 0;
    launch_k<kBlock, k_mask_runs_body>(lc, k_mask_runs, dim3(grid), dim3(kBlock), 0, src, g.nx, g.nrows,
                       g.W, L.S, L.maskbits, L.row_nruns, slice_thr, g.ny, u16_in ? 1 : 0, nt_words);
    timer_end(lc.timer, ST_MASK_RUNS, lc.stream);
    return hipGetLastError();
}

// ----------------------------------------------------------------- runs

// Rows of at most 64 words: lane-per-word.  Each lane finds the runs that
// start in its word; a run still open at the word's end closes at the first
// 0-bit of a later word of the row (segmented suffix minimum across lanes) or
// at nx.  The runs of a step's rows are consecutive in the output, from
// run_off of its first row, and a lane's runs follow those of the lanes
// before it.  A step of many runs (noisy masks: up to 32 a word) is gathered
// in LDS, kStage runs at a time, and written out as contiguous vectors; a
// step of few runs is stored straight from the lanes.
constexpr int kStage = 256;
__device__ __forceinline__ void k_runs_write_lanes_body(const VPart vp, const uint64_t* __restrict__ maskbits, int64_t nx,
                                                             int64_t nrows, int64_t W,
                                                             const uint32_t* __restrict__ run_off,
                                                             uint32_t* __restrict__ xs_out,
                                                             uint32_t* __restrict__ xe_out,
                                                             uint32_t* __restrict__ parent,
                                                             uint32_t* __restrict__ run_row, int64_t row_base,
                                                             const DevState* S) {
    __shared__ uint32_t s_xs[kBlock / kWave][kStage], s_xe[kBlock / kWave][kStage], s_rw[kBlock / kWave][kStage];
    if (thread_exit(S)) return;  // no barrier below; the status is the same for every lane of a wave
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int64_t wave = ((int64_t)vp.b * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)vp.n * blockDim.x / kWave;
    const int64_t R = kWave / W;
    const uint32_t kBig = 0xFFFFFFFFu;
    uint32_t* sx = s_xs[wv];
    uint32_t* se = s_xe[wv];
    uint32_t* sr = s_rw[wv];
    for (int64_t row0 = wave * R; row0 < nrows; row0 += nwaves * R) {
        const WordLane wl = word_lane(row0, W, nrows);
        const uint64_t m = wl.row >= 0 ? maskbits[wl.row * W + wl.w] : 0ull;
        const uint32_t prev_hi = dpp_u32<kDppWaveShr1>(0u, (uint32_t)(m >> 32));
        const uint64_t cin = (wl.w > 0) ? (uint64_t)(prev_hi >> 31) : 0ull;
        const uint64_t starts = m & ~((m << 1) | cin);
        const uint32_t cnt = (uint32_t)__popcll(starts);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t excl = incl - cnt;
        const uint32_t T = (uint32_t)__shfl((int)incl, kWave - 1);
        // first 0-bit position of each word, then the minimum over later words of the row
        uint32_t smin = (wl.row >= 0 && m != ~0ull) ? (uint32_t)(64 * wl.w) + (uint32_t)__ffsll((unsigned long long)~m) - 1u
                                                   : kBig;
        // lane + o lies in this lane's row exactly when lane + o < seg_end
        const int seg_end = wl.seg_first + (int)W;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t other = __shfl_down(smin, o);
            if (lane + o < seg_end) smin = other < smin ? other : smin;
        }
        uint32_t next_zero = __shfl_down(smin, 1);
        if (lane + 1 >= seg_end) next_zero = kBig;
        if (next_zero > (uint32_t)nx) next_zero = (uint32_t)nx;
        if (T == 0) continue;  // uniform
        const uint32_t kb = run_off[row0];  // the step's first run
        const uint32_t rid = (uint32_t)(row_base + wl.row);
        if (T <= (uint32_t)(2 * kWave)) {  // uniform: few runs a lane, stored straight from the lanes
            uint64_t st = starts;
            uint32_t k = kb + excl;
            while (st) {
                const int i = __ffsll((unsigned long long)st) - 1;
                st &= st - 1;
                const uint64_t rest = ~m & (~0ull << i);
                xs_out[k] = (uint32_t)(64 * wl.w + i);
                xe_out[k] = rest ? (uint32_t)(64 * wl.w) + (uint32_t)__ffsll((unsigned long long)rest) - 1u : next_zero;
                parent[k] = k;
                run_row[k] = rid;
                ++k;
            }
            continue;
        }
        for (uint32_t r0 = 0; r0 < T; r0 += (uint32_t)kStage) {
            // this round's runs of the lane into the wave's staging area
            uint64_t st = starts;
            uint32_t k = excl;
            while (st) {
                const int i = __ffsll((unsigned long long)st) - 1;
                st &= st - 1;
                if (k >= r0 + (uint32_t)kStage) break;
                if (k >= r0) {
                    const uint64_t rest = ~m & (~0ull << i);
                    sx[k - r0] = (uint32_t)(64 * wl.w + i);
                    se[k - r0] = rest ? (uint32_t)(64 * wl.w) + (uint32_t)__ffsll((unsigned long long)rest) - 1u : next_zero;
                    sr[k - r0] = rid;
                }
                ++k;
            }
            wave_sync();
            const uint32_t nr = T - r0 < (uint32_t)kStage ? T - r0 : (uint32_t)kStage;
            for (uint32_t j = (uint32_t)lane; j < nr; j += kWave) {
                const uint32_t g = kb + r0 + j;
                xs_out[g] = sx[j];
                xe_out[g] = se[j];
                parent[g] = g;
                run_row[g] = sr[j];
            }
            wave_sync();  // the area is refilled by the next round
        }
    }
}
__global__ __launch_bounds__(kBlock) void k_runs_write_lanes(const uint64_t* __restrict__ maskbits, int64_t nx,
                                                             int64_t nrows, int64_t W,
                                                             const uint32_t* __restrict__ run_off,
                                                             uint32_t* __restrict__ xs_out,
                                                             uint32_t* __restrict__ xe_out,
                                                             uint32_t* __restrict__ parent,
                                                             uint32_t* __restrict__ run_row, int64_t row_base,
                                                             const DevState* S) {
    k_runs_write_lanes_body(hw_part(), maskbits, nx, nrows, W, run_off, xs_out, xe_out, parent, run_row, row_base, S);
}

// Rows of more than 64 words: one thread per row walks the row's words; a
// start event opens a run, an end event (0-bit after a 1-bit) closes it.
__device__ __forceinline__ void k_runs_write_body(const VPart vp, const uint64_t* __restrict__ maskbits, int64_t nrows, int64_t W,
                                                       const uint32_t* __restrict__ run_off, uint32_t* __restrict__ xs_out,
                                                       uint32_t* __restrict__ xe_out, uint32_t* __restrict__ parent,
                                                       uint32_t* __restrict__ run_row, int64_t row_base,
                                                       const DevState* S) {
    if (thread_exit(S)) return;
    const int64_t nthreads = (int64_t)vp.n * blockDim.x;
    for (int64_t row = (int64_t)vp.b * blockDim.x + threadIdx.x; row < nrows; row += nthreads) {
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
                    run_row[k] = (uint32_t)(row_base + row);
                    ++k;
                }
            }
            carry = m >> 63;
        }
        if (carry) {
            xs_out[k] = xs;
            xe_out[k] = (uint32_t)(W * 64);
            parent[k] = k;
            run_row[k] = (uint32_t)(row_base + row);
        }
    }
}
__global__ __launch_bounds__(kBlock) void k_runs_write(const uint64_t* __restrict__ maskbits, int64_t nrows, int64_t W,
                                                       const uint32_t* __restrict__ run_off, uint32_t* __restrict__ xs_out,
                                                       uint32_t* __restrict__ xe_out, uint32_t* __restrict__ parent,
                                                       uint32_t* __restrict__ run_row, int64_t row_base,
                                                       const DevState* S) {
    k_runs_write_body(hw_part(), maskbits, nrows, W, run_off, xs_out, xe_out, parent, run_row, row_base, S);
}

hipError_t launch_runs_write(const LaunchCtx& lc, const Geom& g, const Layout& L, int64_t r0, int64_t r1) {
    timer_begin(lc.timer, ST_RUNS, lc.stream);
    const int64_t nr = r1 - r0;
    const uint64_t* mb = L.maskbits + r0 * g.W;
    const uint32_t* off = L.run_off + r0;
    if (g.W <= kWave) {
        const int64_t R = kWave / g.W;
        launch_k<kBlock, k_runs_write_lanes_body>(lc, k_runs_write_lanes, dim3(grid_for((nr + R - 1) / R, kBlock / kWave, lc.grid_mask)),
                           dim3(kBlock), 0, mb, g.nx, nr, g.W, off, L.run_xs, L.run_xe, L.parent,
                           L.run_row, r0, (const DevState*)L.S);
    } else {
        launch_k<kBlock, k_runs_write_body>(lc, k_runs_write, dim3(grid_for(nr, kBlock, 16384)), dim3(kBlock), 0, mb, nr, g.W,
                           off, L.run_xs, L.run_xe, L.parent, L.run_row, r0, (const DevState*)L.S);
    }
    timer_end(lc.timer, ST_RUNS, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------ union-find

// Root of x with path halving.  Parent pointers only ever point to smaller
// run numbers, so the walk terminates; a halving store only writes an
// ancestor, which is safe against concurrent links (links only change roots).
// Loads go through the per-CU cache and may be stale: any value ever held by
// parent[x] is an ancestor of x, so a stale walk still ends inside x's set,
// and the linking CAS (which sees the current value) decides.  This keeps the
// hot root of a giant component out of a single L2 channel.
__device__ __forceinline__ uint32_t find_root(uint32_t* parent, uint32_t x) {
    while (true) {
        uint32_t p = parent[x];
        if (p == x) return x;
        uint32_t gp = parent[p];
        if (gp == p) return p;
        parent[x] = gp;
        x = gp;
    }
}

__device__ __forceinline__ void unite(uint32_t* parent, uint32_t a, uint32_t b) {
    // same parent (now or at any earlier time) means same set
    if (parent[a] == parent[b]) return;
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

// Union-find in LDS for the runs of one segment (same linking rule).
__device__ __forceinline__ uint32_t lfind(uint32_t* p, uint32_t x) {
    while (true) {
        const uint32_t q = p[x];
        if (q == x) return x;
        const uint32_t g = p[q];
        if (g == q) return q;
        p[x] = g;
        x = g;
    }
}

__device__ __forceinline__ void lunite(uint32_t* p, uint32_t a, uint32_t b) {
    a = lfind(p, a);
    b = lfind(p, b);
    while (a != b) {
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = atomicCAS(&p[b], b, a);
        if (old == b) return;
        b = lfind(p, old);
        a = lfind(p, a);
    }
}

// --------------------------------------------------- run-range segments
//
// The runs are cut into segments of T consecutive run numbers, whatever the
// geometry: a segment may hold several z-planes of a sparse volume or a few
// rows of a dense one, and every workgroup gets the same amount of work.
// Level 1 labels each segment in LDS (all links whose two runs lie in the
// segment, in-plane and across z), level 2 unites the roots of links that
// reach back into an earlier segment in the global forest.

constexpr int kSegCap = 16384;   // runs of a segment labelled in LDS (64 KB)
constexpr int kSegMin = 2048;
constexpr int kSegBlock = 1024;
constexpr int kCrossCap = 4096;  // distinct root pairs per segment head (32 KB)

// T: the launch parameter when set (a multiple of 256 in [256, cap]), else n
// spread over G workgroups, clamped to [kSegMin, cap].  Both levels use the
// same G and cap, so they see the same segments.
__device__ __forceinline__ uint32_t seg_runs(uint32_t n, uint32_t G, uint32_t param, uint32_t cap) {
    if (param) return param;
    uint32_t t = (uint32_t)(((uint64_t)n + G - 1) / G);
    t = (t + 255u) & ~255u;
    return t < (uint32_t)kSegMin ? (uint32_t)kSegMin : (t > cap ? cap : t);
}

// (z, y) of row r = z * ny + y: a double estimate, then an exact correction.
__device__ __forceinline__ void row_zy(uint32_t r, uint32_t ny, double inv_ny, uint32_t& z, uint32_t& y) {
    uint32_t q = (uint32_t)((double)r * inv_ny);
    if ((uint64_t)q * ny > r) --q;
    if ((uint64_t)(q + 1) * ny <= r) ++q;
    z = q;
    y = r - q * ny;
}

// First run b in [b0, b1) of a row that can touch [as, ae): its end reaches
// the start (xe > as for 6-, xe >= as for 26-connectivity).  Runs of a row
// are sorted and disjoint, so the ends increase.
template <bool C26>
__device__ __forceinline__ uint32_t first_touch(const uint32_t* xe, uint32_t b0, uint32_t b1, uint32_t as) {
    while (b0 < b1) {
        const uint32_t mid = b0 + ((b1 - b0) >> 1);
        const uint32_t e = xe[mid];
        if (C26 ? e >= as : e > as)
            b1 = mid;
        else
            b0 = mid + 1;
    }
    return b0;
}

// The rows a run of row r = (z, y) can touch among earlier rows: (z, y-1)
// and (z-1, y), plus (z-1, y-1) and (z-1, y+1) with 26-connectivity (the
// diagonal x steps are in the touch rule).
template <bool C26, typename F>
__device__ __forceinline__ void for_back_rows(uint32_t r, uint32_t z, uint32_t y, uint32_t ny, F&& f) {
    if (y > 0) f(r - 1);
    if (z > 0) {
        const uint32_t rz = r - ny;
        f(rz);
        if (C26) {
            if (y > 0) f(rz - 1);
            if (y + 1 < ny) f(rz + 1);
        }
    }
}

// Level 1: one workgroup per segment [s0, s1).  Thread per run: the touching
// runs of each earlier neighbour row are found by a binary search on their
// ends; pairs inside the segment are united in LDS.  Then parent[run] = the
// run number of its segment-local root.
template <bool C26>
__device__ __forceinline__ void k_seg_label_body(const VPart vp, const uint32_t* __restrict__ run_off,
                                                         const uint32_t* __restrict__ xs,
                                                         const uint32_t* __restrict__ xe,
                                                         const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                         uint32_t ny, double inv_ny, uint32_t G, uint32_t tparam,
                                                         const DevState* S) {
    __shared__ uint32_t lp[kSegCap];
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_runs, lo = S->seg_lo;
    if (n <= lo) return;
    const uint32_t T = seg_runs(n - lo, G, tparam, (uint32_t)kSegCap);
    const uint32_t nseg = (n - lo + T - 1) / T;
    for (uint32_t sg = vp.b; sg < nseg; sg += vp.n) {
        const uint32_t s0 = lo + sg * T, s1 = (n - s0 < T) ? n : s0 + T, m = s1 - s0;
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) lp[i] = i;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            const uint32_t a = s0 + i;
            const uint32_t r = run_row[a];
            uint32_t z, y;
            row_zy(r, ny, inv_ny, z, y);
            const uint32_t as = xs[a], ae = xe[a];
            for_back_rows<C26>(r, z, y, ny, [&](uint32_t rb) {
                uint32_t b0 = run_off[rb];
                const uint32_t b1 = run_off[rb + 1];
                if (b1 <= s0) return;  // the whole row lies in an earlier segment
                if (b0 < s0) b0 = s0;
                for (uint32_t b = first_touch<C26>(xe, b0, b1, as); b < b1; ++b) {
                    const uint32_t bs = xs[b];
                    if (C26 ? bs > ae : bs >= ae) break;
                    lunite(lp, i, b - s0);
                }
            });
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            uint32_t q = i;
            while (lp[q] != q) q = lp[q];
            parent[s0 + i] = s0 + q;
        }
        __syncthreads();  // lp is reused by the next segment
    }
}
template <bool C26>
__global__ __launch_bounds__(kSegBlock) void k_seg_label(const uint32_t* __restrict__ run_off,
                                                         const uint32_t* __restrict__ xs,
                                                         const uint32_t* __restrict__ xe,
                                                         const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                         uint32_t ny, double inv_ny, uint32_t G, uint32_t tparam,
                                                         const DevState* S) {
    k_seg_label_body<C26>(hw_part(), run_off, xs, xe, run_row, parent, ny, inv_ny, G, tparam, S);
}

// Level 2: one workgroup per segment.
// Only runs whose rows lie within ny + 1 rows of the segment's first row can
// touch an earlier segment.  Each touching pair (a, b), b < s0, names the
// pair of their roots; the distinct pairs are collected in an LDS hash set
// (a giant component contributes a handful instead of one per run) and
// united in the global forest.  A full set falls back to direct unions.
template <bool C26>
__device__ __forceinline__ void k_seg_cross_body(const VPart vp, const uint32_t* __restrict__ run_off,
                                                      const uint32_t* __restrict__ xs,
                                                      const uint32_t* __restrict__ xe,
                                                      const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                      uint32_t ny, double inv_ny, int64_t nrows, uint32_t G,
                                                      uint32_t tparam, const DevState* S) {
    __shared__ unsigned long long tab[kCrossCap];
    constexpr unsigned long long kEmpty = ~0ull;
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_runs, lo = S->seg_lo;
    if (n <= lo) return;
    const uint32_t T = seg_runs(n - lo, G, tparam, (uint32_t)kSegCap);
    const uint32_t nseg = (n - lo + T - 1) / T;
    // the very first segment of a volume has nothing before it
    for (uint32_t sg = (lo == 0 ? 1u : 0u) + vp.b; sg < nseg; sg += vp.n) {
        const uint32_t s0 = lo + sg * T, s1 = (n - s0 < T) ? n : s0 + T;
        for (int i = threadIdx.x; i < kCrossCap; i += blockDim.x) tab[i] = kEmpty;
        const uint32_t r0 = run_row[s0];  // rows after r0 hold only runs > s0
        // the head: runs of rows up to r0 + ny + 1 (run rows never decrease
        // with the run number, so a thread stops at its first run past it;
        // offsets of later rows may not exist yet when a volume arrives in slabs)
        const uint64_t rlast = (uint64_t)r0 + ny + 1;
        __syncthreads();
        uint32_t last_a = kNone, last_b = kNone;
        for (uint32_t a = s0 + threadIdx.x; a < s1; a += blockDim.x) {
            const uint32_t r = run_row[a];
            if (r > rlast) break;
            uint32_t z, y;
            row_zy(r, ny, inv_ny, z, y);
            const uint32_t as = xs[a], ae = xe[a];
            uint32_t ra = kNone;
            for_back_rows<C26>(r, z, y, ny, [&](uint32_t rb) {
                if (rb > r0) return;
                const uint32_t b0 = run_off[rb];
                uint32_t b1 = run_off[rb + 1];
                if (b1 > s0) b1 = s0;
                if (b0 >= b1) return;
                for (uint32_t b = first_touch<C26>(xe, b0, b1, as); b < b1; ++b) {
                    const uint32_t bs = xs[b];
                    if (C26 ? bs > ae : bs >= ae) break;
                    if (ra == kNone) ra = parent[a];
                    const uint32_t rbb = parent[b];
                    if (ra == last_a && rbb == last_b) continue;
                    last_a = ra;
                    last_b = rbb;
                    const unsigned long long key = ((unsigned long long)ra << 32) | rbb;
                    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 52) & (kCrossCap - 1);
                    bool done = false;
                    for (int pr = 0; pr < 8; ++pr) {
                        const unsigned long long old = atomicCAS(&tab[h], kEmpty, key);
                        if (old == kEmpty || old == key) {
                            done = true;
                            break;
                        }
                        h = (h + 1) & (kCrossCap - 1);
                    }
                    if (!done) unite(parent, ra, rbb);
                }
            });
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kCrossCap; i += blockDim.x) {
            const unsigned long long key = tab[i];
            if (key != kEmpty) unite(parent, (uint32_t)(key >> 32), (uint32_t)key);
        }
        __syncthreads();  // tab is reused by the next segment
    }
}
template <bool C26>
__global__ __launch_bounds__(kBlock) void k_seg_cross(const uint32_t* __restrict__ run_off,
                                                      const uint32_t* __restrict__ xs,
                                                      const uint32_t* __restrict__ xe,
                                                      const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                      uint32_t ny, double inv_ny, int64_t nrows, uint32_t G,
                                                      uint32_t tparam, const DevState* S) {
    k_seg_cross_body<C26>(hw_part(), run_off, xs, xe, run_row, parent, ny, inv_ny, nrows, G, tparam, S);
}

// ---------------------------------------------- staged (LDS) segment kernels
//
// The same two levels with the data a segment touches copied to LDS first
// (one coalesced pass), so that the binary searches, merges and unions run
// on LDS instead of chains of dependent global loads.  Run extents are
// packed as xs | xe << 16 (rows of at most 65535 voxels).  A segment whose
// rows (or a head whose earlier rows) do not fit the staging arrays reads
// those from global memory instead.

constexpr int kLSeg = 8192;    // runs of a staged segment
constexpr int kLRows = 3072;   // row offsets staged per segment (rows + 1)
constexpr int kHalo = 12288;   // runs of the earlier rows staged for level 2
constexpr int kHaloRows = 3072;

__device__ __forceinline__ uint32_t px(uint32_t v) { return v & 0xFFFFu; }
__device__ __forceinline__ uint32_t pe(uint32_t v) { return v >> 16; }

// first entry of lx[b0, b1) whose end reaches as (the packed form of first_touch)
template <bool C26>
__device__ __forceinline__ uint32_t first_touch_p(const uint32_t* lx, uint32_t b0, uint32_t b1, uint32_t as) {
    while (b0 < b1) {
        const uint32_t mid = b0 + ((b1 - b0) >> 1);
        const uint32_t e = pe(lx[mid]);
        if (C26 ? e >= as : e > as)
            b1 = mid;
        else
            b0 = mid + 1;
    }
    return b0;
}

template <bool C26>
__device__ __forceinline__ void k_seg_label_lds_body(const VPart vp, const uint32_t* __restrict__ run_off,
                                                             const uint32_t* __restrict__ xs,
                                                             const uint32_t* __restrict__ xe,
                                                             const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                             uint32_t ny, double inv_ny, uint32_t G,
                                                             uint32_t tparam, const DevState* S) {
    __shared__ uint32_t lp[kLSeg];
    __shared__ uint32_t lx[kLSeg];
    __shared__ uint32_t loff[kLRows];
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_runs, lo = S->seg_lo;
    if (n <= lo) return;
    const uint32_t T = seg_runs(n - lo, G, tparam, (uint32_t)kLSeg);
    const uint32_t nseg = (n - lo + T - 1) / T;
    for (uint32_t sg = vp.b; sg < nseg; sg += vp.n) {
        const uint32_t s0 = lo + sg * T, s1 = (n - s0 < T) ? n : s0 + T, m = s1 - s0;
        const uint32_t rf = run_row[s0], rl = run_row[s1 - 1];
        const bool rows_in = rl - rf + 2 <= (uint32_t)kLRows;  // offsets of rows rf .. rl + 1
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            lp[i] = i;
            lx[i] = xs[s0 + i] | (xe[s0 + i] << 16);
        }
        if (rows_in)
            for (uint32_t i = threadIdx.x; i < rl - rf + 2; i += blockDim.x) loff[i] = run_off[rf + i];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            const uint32_t r = run_row[s0 + i];
            uint32_t z, y;
            row_zy(r, ny, inv_ny, z, y);
            const uint32_t as = px(lx[i]), ae = pe(lx[i]);
            for_back_rows<C26>(r, z, y, ny, [&](uint32_t rb) {
                if (rb < rf) return;  // rows before the segment's first row hold only earlier runs
                uint32_t b0 = rows_in ? loff[rb - rf] : run_off[rb];
                const uint32_t b1 = rows_in ? loff[rb - rf + 1] : run_off[rb + 1];
                if (b1 <= s0) return;
                if (b0 < s0) b0 = s0;
                for (uint32_t b = first_touch_p<C26>(lx, b0 - s0, b1 - s0, as); b < b1 - s0; ++b) {
                    const uint32_t bs = px(lx[b]);
                    if (C26 ? bs > ae : bs >= ae) break;
                    lunite(lp, i, b);
                }
            });
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            uint32_t q = i;
            while (lp[q] != q) q = lp[q];
            parent[s0 + i] = s0 + q;
        }
        __syncthreads();  // the arrays are reused by the next segment
    }
}
template <bool C26>
__global__ __launch_bounds__(kSegBlock) void k_seg_label_lds(const uint32_t* __restrict__ run_off,
                                                             const uint32_t* __restrict__ xs,
                                                             const uint32_t* __restrict__ xe,
                                                             const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                             uint32_t ny, double inv_ny, uint32_t G,
                                                             uint32_t tparam, const DevState* S) {
    k_seg_label_lds_body<C26>(hw_part(), run_off, xs, xe, run_row, parent, ny, inv_ny, G, tparam, S);
}

template <bool C26>
__device__ __forceinline__ void k_seg_cross_lds_body(const VPart vp, const uint32_t* __restrict__ run_off,
                                                             const uint32_t* __restrict__ xs,
                                                             const uint32_t* __restrict__ xe,
                                                             const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                             uint32_t ny, double inv_ny, uint32_t G,
                                                             uint32_t tparam, const DevState* S) {
    __shared__ unsigned long long tab[kCrossCap];
    __shared__ uint32_t hx[kHalo];
    __shared__ uint32_t hp[kHalo];
    __shared__ uint32_t hoff[kHaloRows];
    constexpr unsigned long long kEmpty = ~0ull;
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_runs, lo = S->seg_lo;
    if (n <= lo) return;
    const uint32_t T = seg_runs(n - lo, G, tparam, (uint32_t)kLSeg);
    const uint32_t nseg = (n - lo + T - 1) / T;
    for (uint32_t sg = (lo == 0 ? 1u : 0u) + vp.b; sg < nseg; sg += vp.n) {
        const uint32_t s0 = lo + sg * T, s1 = (n - s0 < T) ? n : s0 + T;
        for (int i = threadIdx.x; i < kCrossCap; i += blockDim.x) tab[i] = kEmpty;
        const uint32_t r0 = run_row[s0];  // rows after r0 hold only runs > s0
        const uint64_t rlast = (uint64_t)r0 + ny + 1;
        // The halo: the earlier runs a head run (rows r0 .. rh) can reach.
        // Those lie in rows hr0 .. pe of the previous slice (r - ny - 1 ..
        // r - ny + 1) and in rows r0 - 1 and r0 (r - 1).  A head shorter
        // than a slice leaves a gap between the two windows, which is not
        // staged; otherwise they merge into rows hr0 .. r0.
        const uint32_t rh = (uint64_t)run_row[s1 - 1] < rlast ? run_row[s1 - 1] : (uint32_t)rlast;
        const uint32_t hr0 = r0 > ny ? r0 - ny - 1 : 0u;
        const int64_t pe64 = (int64_t)rh + 1 - (int64_t)ny;  // last previous-slice row reached
        const uint32_t sr = r0 > 0 ? r0 - 1 : 0u;             // first same-slice row reached
        const bool gap = pe64 + 1 < (int64_t)sr;
        const uint32_t sS = gap ? sr : r0 + 1;                           // window S: rows sS .. r0
        const int64_t pe = gap ? pe64 : (int64_t)r0;                     // window P: rows hr0 .. pe
        const uint32_t nPr = pe >= (int64_t)hr0 ? (uint32_t)(pe - hr0 + 1) : 0u;  // rows of P
        const uint32_t h0 = run_off[hr0];
        const uint32_t nP = nPr ? (gap ? run_off[hr0 + nPr] : s0) - h0 : 0u;     // runs of P
        const uint32_t hS0 = gap ? run_off[sS] : s0;
        const uint32_t nS = s0 - hS0;                                            // runs of S
        const uint32_t nSr = gap ? r0 - sS + 1 : 0u;
        const bool staged = nP + nS <= (uint32_t)kHalo && nPr + nSr + 2 <= (uint32_t)kHaloRows;
        if (staged) {
            for (uint32_t i = threadIdx.x; i < nP + nS; i += blockDim.x) {
                const uint32_t b = i < nP ? h0 + i : hS0 + (i - nP);
                hx[i] = xs[b] | (xe[b] << 16);
                hp[i] = parent[b];
            }
            for (uint32_t i = threadIdx.x; i < nPr + nSr + 2; i += blockDim.x)
                hoff[i] = i <= nPr ? run_off[hr0 + i] : run_off[sS + (i - nPr - 1)];
        }
        __syncthreads();
        uint32_t last_a = kNone, last_b = kNone;
        for (uint32_t a = s0 + threadIdx.x; a < s1; a += blockDim.x) {
            const uint32_t r = run_row[a];
            if (r > rlast) break;
            uint32_t z, y;
            row_zy(r, ny, inv_ny, z, y);
            const uint32_t as = xs[a], ae = xe[a];
            uint32_t ra = kNone;
            for_back_rows<C26>(r, z, y, ny, [&](uint32_t rb) {
                if (rb > r0) return;
                // staged: run b sits at hx[b - hb]
                uint32_t b0, b1, hb = 0;
                if (!staged) {
                    b0 = run_off[rb];
                    b1 = run_off[rb + 1];
                } else if (rb >= sS) {
                    b0 = hoff[nPr + 1 + (rb - sS)];
                    b1 = hoff[nPr + 2 + (rb - sS)];
                    hb = hS0 - nP;
                } else if ((int64_t)rb <= pe) {
                    b0 = hoff[rb - hr0];
                    b1 = hoff[rb - hr0 + 1];
                    hb = h0;
                } else {
                    return;  // in the gap: no head run reaches it
                }
                if (b1 > s0) b1 = s0;
                if (b0 >= b1) return;
                const uint32_t bb = staged ? first_touch_p<C26>(hx, b0 - hb, b1 - hb, as) + hb
                                           : first_touch<C26>(xe, b0, b1, as);
                for (uint32_t b = bb; b < b1; ++b) {
                    const uint32_t bs = staged ? px(hx[b - hb]) : xs[b];
                    if (C26 ? bs > ae : bs >= ae) break;
                    if (ra == kNone) ra = parent[a];
                    const uint32_t rbb = staged ? hp[b - hb] : parent[b];
                    if (ra == last_a && rbb == last_b) continue;
                    last_a = ra;
                    last_b = rbb;
                    const unsigned long long key = ((unsigned long long)ra << 32) | rbb;
                    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 52) & (kCrossCap - 1);
                    bool done = false;
                    for (int pr = 0; pr < 8; ++pr) {
                        const unsigned long long old = atomicCAS(&tab[h], kEmpty, key);
                        if (old == kEmpty || old == key) {
                            done = true;
                            break;
                        }
                        h = (h + 1) & (kCrossCap - 1);
                    }
                    if (!done) unite(parent, ra, rbb);
                }
            });
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kCrossCap; i += blockDim.x) {
            const unsigned long long key = tab[i];
            if (key != kEmpty) unite(parent, (uint32_t)(key >> 32), (uint32_t)key);
        }
        __syncthreads();  // the arrays are reused by the next segment
    }
}
template <bool C26>
__global__ __launch_bounds__(kSegBlock) void k_seg_cross_lds(const uint32_t* __restrict__ run_off,
                                                             const uint32_t* __restrict__ xs,
                                                             const uint32_t* __restrict__ xe,
                                                             const uint32_t* __restrict__ run_row, uint32_t* parent,
                                                             uint32_t ny, double inv_ny, uint32_t G,
                                                             uint32_t tparam, const DevState* S) {
    k_seg_cross_lds_body<C26>(hw_part(), run_off, xs, xe, run_row, parent, ny, inv_ny, G, tparam, S);
}

hipError_t launch_union(const LaunchCtx& lc, const Geom& g, const Layout& L, int conn) {
    timer_begin(lc.timer, ST_UNION, lc.stream);
    // segments of at least kSegMin runs: a volume planned to hold fewer
    // segments than seg_grid launches one workgroup per planned segment
    const uint32_t G = (uint32_t)runs_grid(g.nrows, kSegMin, lc.seg_grid);
    const uint32_t ny = (uint32_t)g.ny;
    const double inv_ny = 1.0 / (double)g.ny;
    const uint32_t tp = (uint32_t)lc.seg_runs;
    const dim3 grid(G);
    // staged kernels: rows of at most 65535 voxels (packed extents) and
    // segments of at most kLSeg runs
    const bool staged = g.nx <= 65535 && tp <= (uint32_t)kLSeg;
#define SEG_LAUNCH(C)                                                                                           \
    if (staged) {                                                                                               \
        launch_k<kSegBlock, k_seg_label_lds_body<C>>(lc, k_seg_label_lds<C>, grid, dim3(kSegBlock), 0, (const uint32_t*)L.run_off,  \
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, (const uint32_t*)L.run_row,    \
                           L.parent, ny, inv_ny, G, tp, (const DevState*)L.S);                                  \
        launch_k<kSegBlock, k_seg_cross_lds_body<C>>(lc, k_seg_cross_lds<C>, grid, dim3(kSegBlock), 0, (const uint32_t*)L.run_off,  \
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, (const uint32_t*)L.run_row,    \
                           L.parent, ny, inv_ny, G, tp, (const DevState*)L.S);                                  \
    } else {                                                                                                    \
        launch_k<kSegBlock, k_seg_label_body<C>>(lc, k_seg_label<C>, grid, dim3(kSegBlock), 0, (const uint32_t*)L.run_off,      \
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, (const uint32_t*)L.run_row,    \
                           L.parent, ny, inv_ny, G, tp, (const DevState*)L.S);                                  \
        launch_k<kBlock, k_seg_cross_body<C>>(lc, k_seg_cross<C>, grid, dim3(kBlock), 0, (const uint32_t*)L.run_off,         \
                           (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe, (const uint32_t*)L.run_row,    \
                           L.parent, ny, inv_ny, g.nrows, G, tp, (const DevState*)L.S);                         \
    }
    if (conn == 26) {
        SEG_LAUNCH(true)
    } else {
        SEG_LAUNCH(false)
    }
#undef SEG_LAUNCH
    timer_end(lc.timer, ST_UNION, lc.stream);
    return hipGetLastError();
}

// Full compression: parent[i] = root(i); root flags for the component scan.
// The walk only reads: a halving store by one thread could otherwise put an
// intermediate ancestor back into an entry another thread has already set to
// its root.  Each entry is written by its own thread only, so every entry
// ends at its root.
__device__ __forceinline__ void k_flatten_body(const VPart vp, uint32_t* parent, uint32_t* root_flag, const DevState* S) {
    if (thread_exit(S)) return;
    const uint32_t n = S->n_runs;
    const uint32_t nthreads = vp.n * blockDim.x;
    for (uint32_t i = vp.b * blockDim.x + threadIdx.x; i < n; i += nthreads) {
        uint32_t r = i, p = ld_relaxed(&parent[i]);
        while (p != r) {
            r = p;
            p = ld_relaxed(&parent[r]);
        }
        st_relaxed(&parent[i], r);
        root_flag[i] = (r == i) ? 1u : 0u;
    }
}
__global__ __launch_bounds__(kBlock) void k_flatten(uint32_t* parent, uint32_t* root_flag, const DevState* S) {
    k_flatten_body(hw_part(), parent, root_flag, S);
}

hipError_t launch_flatten(const LaunchCtx& lc, const Geom& g, const Layout& L) {
    timer_begin(lc.timer, ST_FLATTEN, lc.stream);
    launch_k<kBlock, k_flatten_body>(lc, k_flatten, dim3(runs_grid(g.nrows, kBlock, lc.grid_stream)), dim3(kBlock), 0,
                       L.parent, L.comp_id,
                       (const DevState*)L.S);
    timer_end(lc.timer, ST_FLATTEN, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------- component stats

constexpr int kStatRuns = 4;     // consecutive runs per thread and round
constexpr int kStatTab = 1024;   // LDS table of component accumulators per workgroup (36 KB)

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

struct StatTab {
    uint32_t key[kStatTab];
    unsigned long long size[kStatTab];
    uint32_t bb[6][kStatTab];
};

// Add an accumulator to the workgroup table (open addressing, a few probes),
// or straight to the component when the table has no room for the root.
__device__ __forceinline__ void tab_add(StatTab& t, uint32_t root, const Acc& a, roix_component* comps,
                                        const uint32_t* comp_id) {
    uint32_t h = (root * 2654435761u) >> 22;  // 10 bits
    for (int pr = 0; pr < 8; ++pr) {
        const uint32_t old = atomicCAS(&t.key[h], kNone, root);
        if (old == kNone || old == root) {
            atomicAdd(&t.size[h], a.size);
            atomicMin(&t.bb[0][h], a.x0);
            atomicMax(&t.bb[1][h], a.x1);
            atomicMin(&t.bb[2][h], a.y0);
            atomicMax(&t.bb[3][h], a.y1);
            atomicMin(&t.bb[4][h], a.z0);
            atomicMax(&t.bb[5][h], a.z1);
            return;
        }
        h = (h + 1) & (kStatTab - 1);
    }
    acc_flush_global(comps, comp_id[root], a);
}

// Called by every lane of the wave: the lanes with `pred` hand in their
// accumulator.  Those that share the first such lane's root (a giant
// component, typically) are reduced across the wave into one table update;
// the others (usually distinct small components) go in one by one.
__device__ __forceinline__ void wave_flush(bool pred, uint32_t root, const Acc& a, StatTab& t, roix_component* comps,
                                           const uint32_t* comp_id) {
    const uint64_t m = __ballot(pred);
    if (!m) return;
    const int lane = threadIdx.x % kWave;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const uint32_t lr = __builtin_amdgcn_readlane(root, leader);
    const bool match = pred && root == lr;
    Acc r;
    r.size = wave_sum(match ? a.size : 0ull);
    r.x0 = wave_min(match ? a.x0 : 0xFFFFFFFFu);
    r.x1 = wave_max(match ? a.x1 : 0u);
    r.y0 = wave_min(match ? a.y0 : 0xFFFFFFFFu);
    r.y1 = wave_max(match ? a.y1 : 0u);
    r.z0 = wave_min(match ? a.z0 : 0xFFFFFFFFu);
    r.z1 = wave_max(match ? a.z1 : 0u);
    if (lane == leader) tab_add(t, lr, r, comps, comp_id);
    if (pred && !match) tab_add(t, root, a, comps, comp_id);
}

// Size and box of every component.  Each workgroup takes a contiguous range
// of runs; a thread accumulates kStatRuns consecutive runs while their root
// stays the same, and hands the accumulator to the workgroup table through
// wave_flush at uniform points.  The table goes to the components once at
// the end, so a giant component costs one set of global atomics per
// workgroup.
__device__ __forceinline__ void k_comp_stats_body(const VPart vp, const uint32_t* __restrict__ xs,
                                                       const uint32_t* __restrict__ xe,
                                                       const uint32_t* __restrict__ run_row,
                                                       const uint32_t* __restrict__ parent,
                                                       const uint32_t* __restrict__ comp_id, uint32_t ny,
                                                       double inv_ny, roix_component* comps, const DevState* S) {
    __shared__ StatTab t;
    for (int i = threadIdx.x; i < kStatTab; i += blockDim.x) {
        t.key[i] = kNone;
        t.size[i] = 0;
        t.bb[0][i] = t.bb[2][i] = t.bb[4][i] = 0xFFFFFFFFu;
        t.bb[1][i] = t.bb[3][i] = t.bb[5][i] = 0u;
    }
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_runs;
    constexpr uint32_t kRound = (uint32_t)kBlock * kStatRuns;
    uint64_t per = ((uint64_t)n + vp.n - 1) / vp.n;
    per = (per + kRound - 1) / kRound * kRound;
    const uint64_t b0 = (uint64_t)vp.b * per;
    const uint64_t b1 = b0 + per < (uint64_t)n ? b0 + per : (uint64_t)n;
    for (uint64_t base = b0; base < b1; base += kRound) {
        const uint64_t i0 = base + (uint64_t)threadIdx.x * kStatRuns;
        uint32_t pr[kStatRuns], sx[kStatRuns], ex[kStatRuns], rw[kStatRuns];
        if (i0 + kStatRuns <= b1) {  // i0 is a multiple of 4: one 16-byte load per array
            const uint4 p4 = *reinterpret_cast<const uint4*>(parent + i0);
            const uint4 s4 = *reinterpret_cast<const uint4*>(xs + i0);
            const uint4 e4 = *reinterpret_cast<const uint4*>(xe + i0);
            const uint4 r4 = *reinterpret_cast<const uint4*>(run_row + i0);
            pr[0] = p4.x, pr[1] = p4.y, pr[2] = p4.z, pr[3] = p4.w;
            sx[0] = s4.x, sx[1] = s4.y, sx[2] = s4.z, sx[3] = s4.w;
            ex[0] = e4.x, ex[1] = e4.y, ex[2] = e4.z, ex[3] = e4.w;
            rw[0] = r4.x, rw[1] = r4.y, rw[2] = r4.z, rw[3] = r4.w;
        } else {
#pragma unroll
            for (int k = 0; k < kStatRuns; ++k) {
                const bool in = i0 + k < b1;
                pr[k] = in ? parent[i0 + k] : kNone;
                sx[k] = in ? xs[i0 + k] : 0u;
                ex[k] = in ? xe[i0 + k] : 0u;
                rw[k] = in ? run_row[i0 + k] : 0u;
            }
        }
        uint32_t cur = kNone;
        Acc a;
        acc_reset(a);
#pragma unroll
        for (int k = 0; k <= kStatRuns; ++k) {
            const uint32_t root = k < kStatRuns ? pr[k] : kNone;
            const bool fl = cur != kNone && root != cur;
            wave_flush(fl, cur, a, t, comps, comp_id);
            if (fl) {
                cur = kNone;
                acc_reset(a);
            }
            if (root != kNone) {
                cur = root;
                uint32_t z, y;
                row_zy(rw[k], ny, inv_ny, z, y);
                a.size += ex[k] - sx[k];
                a.x0 = sx[k] < a.x0 ? sx[k] : a.x0;
                a.x1 = ex[k] > a.x1 ? ex[k] : a.x1;
                a.y0 = y < a.y0 ? y : a.y0;
                a.y1 = y + 1 > a.y1 ? y + 1 : a.y1;
                a.z0 = z < a.z0 ? z : a.z0;
                a.z1 = z + 1 > a.z1 ? z + 1 : a.z1;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kStatTab; i += blockDim.x) {
        const uint32_t key = t.key[i];
        if (key == kNone) continue;
        Acc e;
        e.size = t.size[i];
        e.x0 = t.bb[0][i];
        e.x1 = t.bb[1][i];
        e.y0 = t.bb[2][i];
        e.y1 = t.bb[3][i];
        e.z0 = t.bb[4][i];
        e.z1 = t.bb[5][i];
        acc_flush_global(comps, comp_id[key], e);
    }
}
__global__ __launch_bounds__(kBlock) void k_comp_stats(const uint32_t* __restrict__ xs,
                                                       const uint32_t* __restrict__ xe,
                                                       const uint32_t* __restrict__ run_row,
                                                       const uint32_t* __restrict__ parent,
                                                       const uint32_t* __restrict__ comp_id, uint32_t ny,
                                                       double inv_ny, roix_component* comps, const DevState* S) {
    k_comp_stats_body(hw_part(), xs, xe, run_row, parent, comp_id, ny, inv_ny, comps, S);
}

hipError_t launch_comp_stats(const LaunchCtx& lc, const Geom& g, const Layout& L, roix_component* comps) {
    timer_begin(lc.timer, ST_COMPS, lc.stream);
    launch_k<kBlock, k_comp_stats_body>(lc, k_comp_stats, dim3(runs_grid(g.nrows, kBlock * kStatRuns, lc.stats_grid)),
                       dim3(kBlock), 0, (const uint32_t*)L.run_xs, (const uint32_t*)L.run_xe,
                       (const uint32_t*)L.run_row, (const uint32_t*)L.parent, (const uint32_t*)L.comp_id,
                       (uint32_t)g.ny, 1.0 / (double)g.ny, comps, (const DevState*)L.S);
    timer_end(lc.timer, ST_COMPS, lc.stream);
    return hipGetLastError();
}

// ------------------------------------------------------------- keep rule

// LARGEST in one launch: each workgroup leaves the largest size among its
// components, with the first component holding it, in its slot; the last
// workgroup to finish takes the largest size over the slots (the first
// component on a tie) and keeps that component, and notes its root run.
// Every kept flag was cleared when the component entries were written.
static_assert(kKeepGrid % kBlock == 0, "keep slots per thread");
__device__ __forceinline__ void k_keep_largest_body(const VPart vp, roix_component* comps, uint8_t* kept_flag,
                                                    const uint32_t* __restrict__ run_off,
                                                    const uint32_t* __restrict__ run_xs, int64_t nx, DevState* S) {
    if (block_exit_l(S)) return;  // the status does not change during this launch: every workgroup leaves
    __shared__ unsigned long long s_m[kBlock / kWave];
    __shared__ uint32_t s_c[kBlock / kWave];
    __shared__ int s_last;
    const uint32_t n = S->n_comps;
    unsigned long long m = 0;
    uint32_t best = kNone;
    for (uint32_t c = vp.b * blockDim.x + threadIdx.x; c < n; c += vp.n * blockDim.x) {
        const unsigned long long sz = comps[c].size;
        if (sz > m) {  // c ascending: the first of this thread's largest
            m = sz;
            best = c;
        }
    }
    // (largest size, first component with it) over the workgroup
    const unsigned long long wm = wave_max(m);
    const uint32_t wc = wave_min(m == wm ? best : kNone);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        s_m[w] = wm;
        s_c[w] = wc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bm = 0;
        uint32_t bc = kNone;
        for (int k = 0; k < kBlock / kWave; ++k)
            if (s_m[k] > bm || (s_m[k] == bm && s_c[k] < bc)) {
                bm = s_m[k];
                bc = s_c[k];
            }
        st_dev(&S->keep_size[vp.b], bm);
        st_dev(&S->keep_cid[vp.b], bc);
        wait_mem();  // the slot is in place before the workgroup counts itself done
        s_last = atomicAdd(&S->done_keep, 1u) == vp.n - 1;
    }
    __syncthreads();
    if (!s_last) return;  // uniform
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // the slots, kKeepGrid / kBlock per thread, then across the workgroup
    unsigned long long km[kKeepGrid / kBlock];
    uint32_t kc[kKeepGrid / kBlock];
#pragma unroll
    for (int k = 0; k < kKeepGrid / kBlock; ++k) {
        const uint32_t j = threadIdx.x + (uint32_t)(k * kBlock);
        km[k] = j < vp.n ? ld_dev(&S->keep_size[j]) : 0ull;
        kc[k] = j < vp.n ? ld_dev(&S->keep_cid[j]) : kNone;
    }
    unsigned long long tm = 0;
    uint32_t tc = kNone;
#pragma unroll
    for (int k = 0; k < kKeepGrid / kBlock; ++k)
        if (km[k] > tm || (km[k] == tm && kc[k] < tc)) {
            tm = km[k];
            tc = kc[k];
        }
    const unsigned long long gm = wave_max(tm);
    const uint32_t gc = wave_min(tm == gm ? tc : kNone);
    __syncthreads();  // the per-wave results of the first reduction have been read
    if (threadIdx.x % kWave == 0) {
        s_m[w] = gm;
        s_c[w] = gc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long bm = 0;
    uint32_t bc = kNone;
    for (int k = 0; k < kBlock / kWave; ++k)
        if (s_m[k] > bm || (s_m[k] == bm && s_c[k] < bc)) {
            bm = s_m[k];
            bc = s_c[k];
        }
    S->max_size = bm;
    if (bc == kNone) return;  // no component
    S->largest_cid = bc;
    roix_component* e = comps + bc;
    e->kept = 1u;
    kept_flag[bc] = 1;
    S->n_kept = 1ull;
    S->n_kept_voxels = e->size;
    S->bbox[0] = e->x0;
    S->bbox[1] = e->x1;
    S->bbox[2] = e->y0;
    S->bbox[3] = e->y1;
    S->bbox[4] = e->z0;
    S->bbox[5] = e->z1;
    // its root run: the run of row label / nx that starts at label % nx
    const uint64_t lab = e->label;
    const uint32_t row = (uint32_t)(lab / (uint64_t)nx), x = (uint32_t)(lab % (uint64_t)nx);
    uint32_t a = run_off[row], b = run_off[row + 1];
    while (b - a > 1) {  // runs of a row are in x order
        const uint32_t mid = (a + b) >> 1;
        if (run_xs[mid] <= x)
            a = mid;
        else
            b = mid;
    }
    if (a < run_off[row + 1] && run_xs[a] == x) {
        S->kept_root = a;
        S->kept_by_root = 1u;
    }
}
__global__ __launch_bounds__(kBlock) void k_keep_largest(roix_component* comps, uint8_t* kept_flag,
                                                         const uint32_t* __restrict__ run_off,
                                                         const uint32_t* __restrict__ run_xs, int64_t nx, DevState* S) {
    k_keep_largest_body(hw_part(), comps, kept_flag, run_off, run_xs, nx, S);
}

// kept flags, counts and the union box of kept components
__device__ __forceinline__ void k_keep_apply_body(const VPart vp, roix_component* comps, uint8_t* kept_flag, int largest,
                                                       unsigned long long min_size, DevState* S) {
    if (block_exit_l(S)) return;
    const uint32_t n = S->n_comps;
    const uint32_t lc = S->largest_cid;
    unsigned long long nk = 0, nv = 0;
    uint32_t bb[6] = {0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    for (uint32_t c = vp.b * blockDim.x + threadIdx.x; c < n; c += vp.n * blockDim.x) {
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
__global__ __launch_bounds__(kBlock) void k_keep_apply(roix_component* comps, uint8_t* kept_flag, int largest,
                                                       unsigned long long min_size, DevState* S) {
    k_keep_apply_body(hw_part(), comps, kept_flag, largest, min_size, S);
}

hipError_t launch_keep(const LaunchCtx& lc, const Geom& g, const Layout& L, roix_component* comps,
                       const roix_criterion* crit) {
    timer_begin(lc.timer, ST_KEEP, lc.stream);
    const int grid = runs_grid(g.nrows, kBlock, kKeepGrid);  // components: at most one per run
    if (crit->keep == ROIX_KEEP_LARGEST)
        launch_k<kBlock, k_keep_largest_body>(lc, k_keep_largest, dim3(grid), dim3(kBlock), 0, comps, L.kept_flag,
                                              (const uint32_t*)L.run_off, (const uint32_t*)L.run_xs, g.nx, L.S);
    else
        launch_k<kBlock, k_keep_apply_body>(lc, k_keep_apply, dim3(grid), dim3(kBlock), 0, comps, L.kept_flag, 0,
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
