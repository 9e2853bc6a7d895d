// k_huff.hip - lossless Huffman stage for byte streams (the packed code
// stream, or the output of the paper's quantiser): Huffman coding is among
// the lossless coders the paper lists (Sec. 1).
//
// Code: Huffman's construction over the 256 byte counts with a fixed order
// for equal weights (leaves sorted by (count, byte value) and merged nodes in
// creation order form two queues; each step takes the two lightest heads, a
// leaf before a merged node of the same weight); one used byte gets length 1;
// lengths above 32 are refused.  Canonical codes: within a length, codes
// increase with the byte value, and the first code of a length follows the
// last of the length before, shifted left.
// Format: blocks of 4096 input bytes; block b starts at 32-bit word
// block_off[b] of the payload, its codes one after another from the most
// significant bit of each word down, zero bits to the end of its last word;
// block_off[nblocks] is the payload length in words.
//
// Encoding: a byte histogram (16 copies of LDS counters per workgroup), the
// code built by one workgroup, then a wave per block twice: the block's bit
// count (for an exclusive scan of the block sizes), and the codes, ORed into
// the block's words in an LDS window at the positions a wave prefix sum
// gives, then copied out.
// Decoding: a lane per block with a 64-bit bit window fed a 16-byte load
// ahead, an 11-bit lookup table that yields one or two codes, and a
// canonical search for longer codes.
#include "common.h"

namespace roix {

constexpr int kHfBlock = 4096;   // input bytes per block
constexpr int kHfPeek = 11;      // bits of the decoder's lookup table
constexpr int kHfRound = 8;      // decoder steps between refills (2 bytes each at most)
constexpr int kHfRing = 36;      // LDS bytes of a lane's 32-byte output ring (stride against bank conflicts)
constexpr int kHf3Peek = 12;     // bits of the three-code lookup table of the sub-block decoder
constexpr int kHf3Round = 5;     // its steps between refills (3 bytes each at most: 15 bytes a round)
constexpr int kHfSub = 256;      // input bytes per sub-block of the sub-block index
constexpr int kHfSubs = kHfBlock / kHfSub;

struct HfState {
    unsigned long long hist[256];
    uint32_t code[256];
    uint8_t len[256];
    int32_t status;
    int32_t max_len;
};

// ------------------------------------------------------------ histogram

__global__ __launch_bounds__(256) void k_hf_clear(HfState* S) {
    S->hist[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        S->status = 0;
        S->max_len = 0;
    }
}

// 16 copies of the 256 counters per workgroup, lane l adding to copy l % 16:
// lanes that hold the same byte value collide 16 times less often (skewed
// streams, such as the high bytes of wide codes, have few hot values)
constexpr int kHfCopies = 16;

__global__ __launch_bounds__(256) void k_hf_hist(const uint8_t* __restrict__ in, unsigned long long n, HfState* S) {
    __shared__ uint32_t h[256 * kHfCopies];
    for (int i = threadIdx.x; i < 256 * kHfCopies; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const uint32_t copy = threadIdx.x % kHfCopies;
    const unsigned long long nv = n / 16;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const uint4 v = ld_stream(reinterpret_cast<const uint4*>(in) + i);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) atomicAdd(&h[((w[k >> 2] >> (8 * (k & 3))) & 0xFFu) * kHfCopies + copy], 1u);
    }
    // the tail of fewer than 16 bytes
    if (blockIdx.x == 0)
        for (unsigned long long i = nv * 16 + threadIdx.x; i < n; i += blockDim.x)
            atomicAdd(&h[(uint32_t)in[i] * kHfCopies + copy], 1u);
    __syncthreads();
    uint32_t sum = 0u;
#pragma unroll
    for (int c = 0; c < kHfCopies; ++c) sum += h[threadIdx.x * kHfCopies + c];
    if (sum) atomicAdd(&S->hist[threadIdx.x], (unsigned long long)sum);
}

// ------------------------------------------------------------ the code

__global__ __launch_bounds__(256) void k_hf_build(HfState* S, uint8_t* lengths_out) {
    __shared__ unsigned long long w[511];
    __shared__ int parent[511];
    __shared__ int sym[256];
    __shared__ int ns_sh, maxl_sh, bad_sh;
    __shared__ uint32_t bl_count[34], next_code[34];
    __shared__ unsigned long long hs[256];
    __shared__ uint8_t lens[256];
    const int t = threadIdx.x;
    const unsigned long long c = S->hist[t];
    hs[t] = c;
    // rank of this byte among the used ones by (count, byte value)
    if (t == 0) {
        ns_sh = 0;
        maxl_sh = 0;
        bad_sh = 0;
    }
    if (t < 34) bl_count[t] = 0u;
    __syncthreads();
    if (c) atomicAdd(&ns_sh, 1);
    int rank = 0;
    for (int u = 0; u < 256; ++u) {
        const unsigned long long cu = hs[u];
        rank += (cu && (cu < c || (cu == c && u < t))) ? 1 : 0;
    }
    __syncthreads();
    if (c) sym[rank] = t;
    __syncthreads();
    const int ns = ns_sh;
    if (t < ns) w[t] = hs[sym[t]];  // the leaves, lightest first
    __syncthreads();
    // the two-queue merge (sequential: each step depends on the last); the
    // heads of both queues stay in registers, lw = w[lq] and, while the
    // merged queue is not empty (mq < next), mw = w[mq]
    if (t == 0 && ns > 1) {
        int lq = 0, mq = ns, next = ns;
        unsigned long long lw = w[0], mw = 0ull;
        while (next < 2 * ns - 1) {
            int p[2];
            unsigned long long sum = 0ull;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (lq < ns && (mq >= next || lw <= mw)) {  // a leaf before a merged node of the same weight
                    p[k] = lq++;
                    sum += lw;
                    lw = lq < ns ? w[lq] : 0ull;
                } else {
                    p[k] = mq++;
                    sum += mw;
                    mw = mq < next ? w[mq] : 0ull;
                }
            }
            w[next] = sum;
            if (mq == next) mw = sum;  // the merged queue was empty: the new node heads it
            parent[p[0]] = next;
            parent[p[1]] = next;
            ++next;
        }
    }
    __syncthreads();
    // a leaf's code length is its depth: the steps from it up to the root
    int len = 0;
    if (c) {
        if (ns == 1) {
            len = 1;
        } else {
            for (int v = rank; v != 2 * ns - 2; v = parent[v]) ++len;
        }
        atomicMax(&maxl_sh, len);
        if (len > 32) {
            bad_sh = 1;
            len = 0;
        }
    }
    lens[t] = (uint8_t)len;
    if (len) atomicAdd(&bl_count[len], 1u);
    __syncthreads();
    if (t == 0) {  // canonical codes: the first code of each length
        S->max_len = maxl_sh;
        if (bad_sh) S->status = ROIX_ERANGE;
        unsigned long long cc = 0ull;
        next_code[0] = 0u;
        for (int b = 1; b <= 32; ++b) {
            cc = (cc + (b > 1 ? bl_count[b - 1] : 0u)) << 1;
            next_code[b] = (uint32_t)cc;
        }
    }
    __syncthreads();
    // within a length, codes follow the byte values
    uint32_t code = 0u;
    if (len) {
        uint32_t r = 0u;
        for (int u = 0; u < t; ++u) r += lens[u] == len ? 1u : 0u;
        code = next_code[len] + r;
    }
    S->len[t] = (uint8_t)len;
    S->code[t] = code;
    if (lengths_out) lengths_out[t] = (uint8_t)len;
}

// ------------------------------------------------------------ encoding

// Bit count of each block: lane l takes bytes 1024 i + 16 l .. + 15 of the
// block (i = 0..3), so each load instruction reads 1 KB contiguously.
__global__ __launch_bounds__(kWave) void k_hf_count(const uint8_t* __restrict__ in, unsigned long long n,
                                                    const HfState* S, unsigned long long* block_words,
                                                    uint16_t* sub_bits) {
    __shared__ uint8_t len[256];
    for (int i = threadIdx.x; i < 256; i += kWave) len[i] = S->len[i];
    __syncthreads();
    const int lane = threadIdx.x;
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    for (unsigned long long b = blockIdx.x; b < nb; b += gridDim.x) {
        uint4 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned long long p = b * kHfBlock + 1024ull * i + 16ull * lane;
            if (p + 16 <= n) {
                v[i] = ld_stream(reinterpret_cast<const uint4*>(in + p));
            } else {  // the stream's last bytes
                uint32_t w4[4] = {0u, 0u, 0u, 0u};
                for (int k = 0; k < 16; ++k)
                    if (p + k < n) w4[k >> 2] |= (uint32_t)in[p + k] << (8 * (k & 3));
                v[i] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
            }
        }
        uint32_t bits = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned long long p = b * kHfBlock + 1024ull * i + 16ull * lane;
            const int cnt = p >= n ? 0 : (n - p >= 16 ? 16 : (int)(n - p));
            const uint32_t ww[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
            uint32_t bi = 0u;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < cnt) bi += len[(ww[k >> 2] >> (8 * (k & 3))) & 0xFFu];
            bits += bi;
            if (sub_bits) {  // uniform: sub-block 4 i + l / 16 is lanes l / 16 * 16 .. + 15 of step i
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) bi += __shfl_xor(bi, o);
                if ((lane & 15) == 0) sub_bits[b * kHfSubs + 4 * i + lane / 16] = (uint16_t)bi;
            }
        }
        bits = wave_sum(bits);
        if (lane == 0) block_words[b] = (bits + 31u) / 32u;
    }
}

// One lane's 32 bytes of a half block, emitted into the window [pb, pb + nw)
// of the block's output words: the lane's bits [pos, pos + bits) gather in
// a 64-bit accumulator (acc_n bits, most significant first) and the words
// that fall in the window are written; a lane's interior words are its own
// (plain LDS stores), its first and last may be shared with the neighbours
// (ORed).  e[k]: the table entry of byte k, code << 6 | length when P, the
// length alone otherwise (the code then read again by the byte in q).
template <bool P>
__device__ __forceinline__ void hf_emit_half(const uint32_t (&e)[32], const uint4 (&q)[2], int cnt, uint32_t pos,
                                             uint32_t bits, uint32_t pb, uint32_t nw, const uint32_t* code,
                                             uint32_t* buf) {
    const uint32_t first_w = pos >> 5, last_w = (pos + bits - 1u) >> 5;
    if (bits == 0u || last_w < pb || first_w >= pb + nw) return;
    const uint32_t ww[8] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w};
    unsigned long long acc = 0ull;
    uint32_t acc_n = pos & 31u;  // the word starts before the lane's first bit: zeros there
    uint32_t wi = first_w;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k < cnt) {
            const uint32_t L = P ? (e[k] & 63u) : e[k];
            const uint32_t c = P ? (e[k] >> 6) : code[(ww[k >> 2] >> (8 * (k & 3))) & 0xFFu];
            acc |= (unsigned long long)c << (64u - acc_n - L);
            acc_n += L;
            if (acc_n >= 32u) {
                const uint32_t word = (uint32_t)(acc >> 32);
                const uint32_t r = wi - pb;
                if (r < nw) {
                    if (wi == first_w || wi == last_w) atomicOr(&buf[r], word);
                    else buf[r] = word;
                }
                ++wi;
                acc <<= 32;
                acc_n -= 32u;
            }
        }
    }
    if (acc_n > 0u && wi - pb < nw) atomicOr(&buf[wi - pb], (uint32_t)(acc >> 32));
}

// Half h of block b in one window: lane l takes bytes 2048 h + 32 l ..
// + 31, so a half is 2 KB read contiguously and its bits follow the lanes in
// order.  Returns the half's bit count.
template <bool P>
__device__ __forceinline__ uint32_t hf_half(const uint8_t* __restrict__ in, unsigned long long n,
                                            unsigned long long p0, uint32_t carry, uint32_t pb, uint32_t nw,
                                            const uint32_t* tab, const uint32_t* code, uint32_t* buf) {
    const int lane = threadIdx.x;
    const unsigned long long p = p0 + 32ull * lane;
    const int cnt = p >= n ? 0 : (n - p >= 32 ? 32 : (int)(n - p));
    uint4 q[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const unsigned long long pi = p + 16ull * i;
        if (pi + 16 <= n) {
            q[i] = *reinterpret_cast<const uint4*>(in + pi);
        } else {
            uint32_t w4[4] = {0u, 0u, 0u, 0u};
            for (int k = 0; k < 16; ++k)
                if (pi + k < n) w4[k >> 2] |= (uint32_t)in[pi + k] << (8 * (k & 3));
            q[i] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
        }
    }
    const uint32_t ww[8] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w};
    uint32_t e[32];
    uint32_t bits = 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        e[k] = k < cnt ? tab[(ww[k >> 2] >> (8 * (k & 3))) & 0xFFu] : 0u;
        bits += P ? (e[k] & 63u) : e[k];
    }
    // inclusive prefix of the lanes' bit counts
    uint32_t inc = bits;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    hf_emit_half<P>(e, q, cnt, carry + inc - bits, bits, pb, nw, code, buf);
    return (uint32_t)__shfl(inc, kWave - 1);
}

// A wave per block: each half's table entries, bit counts and their prefix,
// then the codes ORed into the block's words in LDS and copied out.  The
// LDS window holds kHfBufWords words (8 bits a byte); a block that needs
// more (long codes) goes through it in several windows.
constexpr uint32_t kHfBufWords = 1024;

__global__ __launch_bounds__(kWave) void k_hf_encode(const uint8_t* __restrict__ in, unsigned long long n,
                                                     const HfState* S, const unsigned long long* block_off,
                                                     uint32_t* __restrict__ payload, unsigned long long cap_words) {
    __shared__ uint32_t code[256];
    __shared__ uint32_t tab[256];  // code << 6 | length when every length is at most 26, else the length
    __shared__ uint32_t buf[kHfBufWords];
    const int lane = threadIdx.x;
    const bool packed = S->max_len <= 26;  // uniform
    for (int i = lane; i < 256; i += kWave) {
        const uint32_t L = S->len[i], c = S->code[i];
        code[i] = c;
        tab[i] = packed ? (c << 6) | L : L;
    }
    __syncthreads();
    if (S->status != 0) return;
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    for (unsigned long long b = blockIdx.x; b < nb; b += gridDim.x) {
        const unsigned long long w0 = block_off[b], w1 = block_off[b + 1];
        if (w1 > cap_words) continue;  // the payload does not hold this block (reported as ETRUNC)
        const uint32_t words = (uint32_t)(w1 - w0);
        for (uint32_t pb = 0; pb < words; pb += kHfBufWords) {
            const uint32_t nw = words - pb < kHfBufWords ? words - pb : kHfBufWords;
            __syncthreads();  // the last window's copy is done
            for (uint32_t i = lane; i < nw; i += kWave) buf[i] = 0u;
            __syncthreads();
            uint32_t carry = 0u;
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                const unsigned long long p0 = b * kHfBlock + (unsigned long long)h * (kHfBlock / 2);
                carry += packed ? hf_half<true>(in, n, p0, carry, pb, nw, tab, code, buf)
                                : hf_half<false>(in, n, p0, carry, pb, nw, tab, code, buf);
            }
            __syncthreads();
            for (uint32_t i = lane; i < nw; i += kWave) payload[w0 + pb + i] = buf[i];
        }
    }
}

__global__ void k_hf_zero_off(unsigned long long* block_off) { block_off[0] = 0ull; }

__global__ void k_hf_finalize(const HfState* S, const unsigned long long* block_off, unsigned long long n,
                              unsigned long long cap_words, int with_sub, roix_huff_info* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    const unsigned long long words = block_off[nb];
    int32_t st = S->status;
    if (st == 0 && words > cap_words) st = ROIX_ETRUNC;
    info->status = st;
    info->max_len = S->max_len;
    info->n = n;
    info->n_blocks = nb;
    info->payload_words = words;
    info->compressed_bytes = 256ull + 8ull * (nb + 1) + 4ull * words + (with_sub ? 2ull * kHfSubs * nb : 0ull);
    info->pad[0] = info->pad[1] = info->pad[2] = 0ull;
}

// ------------------------------------------------------------ decoding

// Decoder tables, built in LDS by each workgroup.  The lookup entry of the
// next kHfPeek bits holds the first code's byte and length (bits 0-7,
// 16-20) and, when a second whole code follows inside the same kHfPeek
// bits, that one's byte and length (bits 8-15, 21-25; length 0: none).
// A first length of 0 marks a code longer than the table.
template <int PK>
struct HfDecodeP {
    uint32_t first[34];   // first canonical code of each length
    uint32_t count[34];   // codes of each length
    uint32_t index[34];   // position of a length's first byte in sym
    uint8_t sym[256];     // bytes by (length, value)
    uint32_t peek[1 << PK];
    int maxl;             // longest code length in use
};
using HfDecode = HfDecodeP<kHfPeek>;

// The code of length <= lmax at the top of the PK-bit value e (canonical: a
// length-L code c is valid when c - first[L] < count[L]).
template <int PK>
__device__ __forceinline__ bool hf_short_code(const HfDecodeP<PK>& T, uint32_t e, int lmax, int& L, uint32_t& s) {
#pragma unroll 1
    for (L = 1; L <= lmax; ++L) {
        const uint32_t c = e >> (PK - L);
        if (c - T.first[L] < T.count[L]) {
            s = T.sym[T.index[L] + (c - T.first[L])];
            return true;
        }
    }
    return false;
}

// Four payload words from quad-aligned word a; words at or past w1 read as
// zero (they are never consumed) and the quad is one 16-byte load when the
// payload is 16-byte aligned and the quad lies inside it.
__device__ __forceinline__ void hf_quad(const uint32_t* __restrict__ payload, unsigned long long a,
                                        unsigned long long w1, unsigned long long pw, bool vec, uint32_t (&q)[4]) {
    if (vec && a + 4 <= pw) {
        const uint4 v = *reinterpret_cast<const uint4*>(payload + a);
        q[0] = v.x;
        q[1] = v.y;
        q[2] = v.z;
        q[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = a + k < w1 ? payload[a + k] : 0u;
    }
}

// The decoder tables of one workgroup (lookup table, canonical bounds),
// built in LDS from the 256 code lengths; false (and EINVAL in S) when the
// lengths are no prefix code.  Every thread of the workgroup calls it.
template <int PK>
__device__ __forceinline__ bool hf_tables(const uint8_t* lengths, unsigned long long n, HfDecodeP<PK>& T, HfState* S) {
    __shared__ int bad_table;
    __shared__ unsigned long long kraft;  // in units of 2^-32
    __shared__ uint8_t lens[256];
    const int t = threadIdx.x;
    const int Lt = lengths[t];
    lens[t] = (uint8_t)Lt;
    if (t < 34) T.count[t] = 0u;
    if (t == 0) {
        bad_table = 0;
        kraft = 0ull;
    }
    __syncthreads();
    if (Lt > 32) bad_table = 1;
    else if (Lt) {
        atomicAdd(&T.count[Lt], 1u);
        atomicAdd(&kraft, 1ull << (32 - Lt));
    }
    __syncthreads();
    if (t == 0) {
        if (kraft > (1ull << 32) || (n > 0 && kraft == 0ull)) bad_table = 1;
        uint32_t pos = 0u;
        unsigned long long c = 0ull;
        T.count[0] = 0u;
        for (int L = 1; L <= 32; ++L) {
            c = (c + T.count[L - 1]) << 1;
            T.first[L] = (uint32_t)c;
            T.index[L] = pos;
            pos += T.count[L];
        }
        T.first[0] = T.index[0] = 0u;
        T.first[33] = T.count[33] = T.index[33] = 0u;
        int ml = 0;
        for (int L = 1; L <= 32; ++L) ml = T.count[L] ? L : ml;
        T.maxl = ml;
    }
    __syncthreads();
    if (Lt >= 1 && Lt <= 32) {  // byte t's place among the bytes of its length
        uint32_t r = 0u;
        for (int u = 0; u < t; ++u) r += lens[u] == Lt ? 1u : 0u;
        T.sym[T.index[Lt] + r] = (uint8_t)t;
    }
    __syncthreads();
    if (bad_table) {
        if (t == 0) atomicCAS(&S->status, 0, ROIX_EINVAL);
        return false;
    }
    for (int e = t; e < (1 << PK); e += blockDim.x) {
        uint32_t val = 0u, s1 = 0u, s2 = 0u;
        int L1 = 0, L2 = 0;
        if (hf_short_code<PK>(T, (uint32_t)e, PK, L1, s1)) {
            val = s1 | ((uint32_t)L1 << 16);
            if (L1 < PK && hf_short_code<PK>(T, ((uint32_t)e << L1) & ((1u << PK) - 1u), PK - L1, L2, s2))
                val |= (s2 << 8) | ((uint32_t)L2 << 21);
        }
        T.peek[e] = val;
    }
    __syncthreads();
    return true;
}

// The three-code lookup table of the sub-block decoder: entry e holds the
// whole codes that start at the top of the kHf3Peek-bit value e, up to three
// of them: their bytes (bits 0-23, the first code's lowest), their total
// length (bits 24-27) and their count (bits 28-29; 0 when the first code is
// longer than the table).  One thread per entry; each workgroup first builds
// the canonical bounds (hf_tables also checks the lengths).
__global__ __launch_bounds__(256) void k_hf_peek3(const uint8_t* lengths, unsigned long long n, uint32_t* tab,
                                                  HfState* S) {
    __shared__ HfDecode T;
    if (!hf_tables<kHfPeek>(lengths, n, T, S)) return;
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (1u << kHf3Peek)) return;
    uint32_t bytes = 0u, tot = 0u, cnt = 0u;
    while (cnt < 3u) {
        const uint32_t room = (uint32_t)kHf3Peek - tot;
        uint32_t L = 1u, sym = 0u;
        bool found = false;
        for (; L <= room; ++L) {
            const uint32_t c = (e >> (room - L)) & ((1u << L) - 1u);
            if (c - T.first[L] < T.count[L]) {
                sym = T.sym[T.index[L] + (c - T.first[L])];
                found = true;
                break;
            }
        }
        if (!found) break;
        bytes |= sym << (8u * cnt);
        tot += L;
        ++cnt;
    }
    tab[e] = bytes | (tot << 24) | (cnt << 28);
}

// A lane decodes one task: a whole block (SUB false), or with the sub-block
// index one 256-byte sub-block (SUB true: 16 lanes per block, each starting
// at the bit the index gives, so that a wave decodes 4 blocks at once).
// Lanes keep a 64-bit bit window fed from 16-byte loads one quad ahead; an
// 11-bit lookup table yields one or two codes, a canonical search the longer
// ones.  A sub-block must take exactly its stated bits.
// P3 (with SUB): each step first looks up the next kHf3Peek bits in the
// three-code table tab3 (staged in LDS), and takes up to three codes at once
// when they all belong to the task and lie in the window; otherwise one code
// as above.  Rounds are then kHf3Round steps, so that the ring never holds
// more than 31 bytes.
template <bool SUB, bool P3 = false>
__global__ __launch_bounds__(256) void k_hf_decode(const uint8_t* lengths, const unsigned long long* block_off,
                                                   const uint16_t* sub_bits, const uint32_t* payload,
                                                   unsigned long long payload_words, unsigned long long n,
                                                   uint8_t* out, HfState* S, int vec, const uint32_t* tab3) {
    __shared__ HfDecode T;
    __shared__ __align__(16) uint8_t ring_sh[kHfRing * 256];
    __shared__ __align__(16) uint32_t P3t[P3 ? (1 << kHf3Peek) : 4];
    if (!hf_tables<kHfPeek>(lengths, n, T, S)) return;
    const int t = threadIdx.x;
    if constexpr (P3) {
        for (int i = t; i < (1 << kHf3Peek) / 4; i += blockDim.x)
            reinterpret_cast<uint4*>(P3t)[i] = reinterpret_cast<const uint4*>(tab3)[i];
        __syncthreads();
    }
    constexpr int kSteps = P3 ? kHf3Round : kHfRound;
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    const unsigned long long ntasks = SUB ? nb * kHfSubs : nb;
    const int maxl = T.maxl;
    // with words still outside the window, a step decodes only when this many
    // bits are in it (a code of the longest length; the three-code table's bits)
    const int need = P3 && maxl < kHf3Peek ? kHf3Peek : maxl;
    uint8_t* ring = ring_sh + kHfRing * t;  // this lane's output bytes, 16 at a time to HBM
    // The wave goes in rounds: at the top of a round each lane takes the
    // quad it loaded the round before, asks for the next, and stores 16
    // output bytes; then kHfRound steps decode from registers only (a lane
    // whose bits run short before its next quad arrives waits a round).
    for (unsigned long long base = (unsigned long long)blockIdx.x * blockDim.x; base < ntasks;
         base += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long task = base + t;
        bool live = task < ntasks;
        const unsigned long long b = SUB ? task / kHfSubs : task;
        unsigned long long w0 = 0ull, w1 = 0ull;
        if (live) {
            w0 = block_off[b];
            w1 = block_off[b + 1];
            if ((b == 0 && w0 != 0) || w1 < w0 || w1 > payload_words) {
                atomicCAS(&S->status, 0, ROIX_EINVAL);
                live = false;
            }
        }
        // the task's bytes [i0, i0 + left) and payload bits [bit0, bit0 + sb)
        unsigned long long i0 = b * kHfBlock, bit0 = 32ull * w0, wa = w0, wend = w1;
        uint32_t sb = 0u;
        if (SUB) {
            i0 += (unsigned long long)(task % kHfSubs) * kHfSub;
            sb = live ? (uint32_t)sub_bits[task] : 0u;
            // the sub-block's start: the stated bits of the block's sub-blocks
            // before it (a scan over its 16 lanes, every lane taking part)
            uint32_t incl = sb;
#pragma unroll
            for (int o = 1; o < kHfSubs; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, kHfSubs);
                if ((t & (kHfSubs - 1)) >= o) incl += y;
            }
            const uint32_t total = __shfl(incl, kHfSubs - 1, kHfSubs);
            if (live && total > 32ull * (w1 - w0)) {
                atomicCAS(&S->status, 0, ROIX_EINVAL);
                live = false;
            }
            bit0 += incl - sb;
            wa = bit0 / 32ull;
            wend = (bit0 + sb + 31ull) / 32ull;
        }
        const unsigned long long iend = SUB ? i0 + kHfSub : i0 + kHfBlock;
        uint32_t left = live && i0 < n ? (uint32_t)((iend < n ? iend : n) - i0) : 0u;  // bytes to decode
        uint32_t rem = live ? (uint32_t)(wend - wa) : 0u;  // payload words not yet in the window
        // quad A holds payload words qa..qa+3 (the next one to take: ci),
        // quad B the four after it once valid, Lq the quad in flight
        unsigned long long qa = wa & ~3ull;
        uint32_t ci = (uint32_t)(wa & 3ull);
        uint32_t A[4] = {0u, 0u, 0u, 0u}, B[4] = {0u, 0u, 0u, 0u}, Lq[4] = {0u, 0u, 0u, 0u};
        bool bvalid = false, pending = false;
        if (live && rem > 0u) hf_quad(payload, qa, wend, payload_words, vec, A);
        // A arrives here: the steps below then wait on nothing but LDS
        __builtin_amdgcn_s_waitcnt(0);
        unsigned long long window = 0ull;  // bits, the next one most significant
        int have = 0;
        if (SUB && rem > 0u) {  // the first word, less the bits before the sub-block
            const uint32_t word = ci == 0u ? A[0] : ci == 1u ? A[1] : ci == 2u ? A[2] : A[3];
            const int skip = (int)(bit0 & 31ull);
            window = ((unsigned long long)word << 32) << skip;
            have = 32 - skip;
            ci += 1u;
            rem -= 1u;
        }
        bool ok = true;
        uint32_t used = 0u;             // bits the task's codes took
        uint32_t wr = 0u, rd = 0u;      // ring bytes written, stored
        unsigned long long g = i0;      // output position of the next store
        while (__any(ok && left > 0u)) {
            if (pending) {
#pragma unroll
                for (int k = 0; k < 4; ++k) B[k] = Lq[k];
                bvalid = true;
                pending = false;
            }
            if (ci == 4u && bvalid) {
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = B[k];
                ci = 0u;
                qa += 4;
                bvalid = false;
            }
            if (!bvalid && rem > 4u - ci) {  // words past quad A
                hf_quad(payload, qa + 4, wend, payload_words, vec, Lq);
                pending = true;
            }
            if (wr - rd >= 16u) {
                const uint32_t* r32 = reinterpret_cast<const uint32_t*>(ring + (rd & 31u));
                *reinterpret_cast<uint4*>(out + g) = make_uint4(r32[0], r32[1], r32[2], r32[3]);
                g += 16;
                rd += 16u;
            }
#pragma unroll 1
            for (int it = 0; it < kSteps; ++it) {
                // take a word into the window (no branch)
                const bool take = have <= 32 && ci < 4u && rem > 0u;
                const uint32_t word = ci == 0u ? A[0] : ci == 1u ? A[1] : ci == 2u ? A[2] : A[3];
                const unsigned long long add = (unsigned long long)word << ((32 - have) & 63);
                window |= take ? add : 0ull;
                have += take ? 32 : 0;
                ci += take ? 1u : 0u;
                rem -= take ? 1u : 0u;
                const bool shift = ci == 4u && bvalid;
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = shift ? B[k] : A[k];
                ci = shift ? 0u : ci;
                qa += shift ? 4ull : 0ull;
                bvalid = bvalid && !shift;
                // with words still outside the window, decode only what is sure to fit
                if (!ok || left == 0u || (rem > 0u && have < need)) continue;
                if constexpr (P3) {
                    const uint32_t e3 = P3t[window >> (64 - kHf3Peek)];
                    const uint32_t c3 = e3 >> 28, L3 = (e3 >> 24) & 15u;
                    if (c3 != 0u && c3 <= left && (int)L3 <= have) {  // up to three codes of the task
                        window <<= L3;
                        have -= (int)L3;
                        used += L3;
                        // all three bytes always: those past the codes' count land
                        // past the ring's live bytes and are overwritten later
                        ring[wr & 31u] = (uint8_t)e3;
                        ring[(wr + 1u) & 31u] = (uint8_t)(e3 >> 8);
                        ring[(wr + 2u) & 31u] = (uint8_t)(e3 >> 16);
                        wr += c3;
                        left -= c3;
                        continue;
                    }
                }
                const uint32_t pk = T.peek[window >> (64 - kHfPeek)];
                int L = (int)((pk >> 16) & 31u);
                uint32_t v = pk;
                if (L == 0) {  // a code longer than the table
                    for (L = kHfPeek + 1; L <= 32; ++L) {  // L = 33 after the loop: no code
                        const uint32_t c = (uint32_t)(window >> (64 - L));
                        if (c - T.first[L] < T.count[L]) {
                            v = T.sym[T.index[L] + (c - T.first[L])];
                            break;
                        }
                    }
                }
                const int L2 = (int)(pk >> 21);
                const bool pair = L2 != 0 && left > 1u && L + L2 <= have;
                L += pair ? L2 : 0;
                const uint32_t k = pair ? 2u : 1u;
                if (L > 32 || L > have) {  // no code, or past the task's payload
                    ok = false;
                    continue;
                }
                window <<= L;
                have -= L;
                used += (uint32_t)L;
                // both bytes always: a second byte of a single code lands
                // past the ring's live bytes and is overwritten later
                ring[wr & 31u] = (uint8_t)v;
                ring[(wr + 1u) & 31u] = (uint8_t)(v >> 8);
                wr += k;
                left -= k;
            }
        }
        if (!live) continue;
        if (!ok || (SUB && used != sb)) {
            atomicCAS(&S->status, 0, ROIX_EINVAL);
            continue;
        }
        if (wr - rd >= 16u) {
            const uint32_t* r32 = reinterpret_cast<const uint32_t*>(ring + (rd & 31u));
            *reinterpret_cast<uint4*>(out + g) = make_uint4(r32[0], r32[1], r32[2], r32[3]);
            g += 16;
            rd += 16u;
        }
        for (uint32_t k = rd; k < wr; ++k) out[g + (k - rd)] = ring[k & 31u];  // the task's last bytes
    }
}

__global__ void k_hf_decode_finalize(const HfState* S, unsigned long long n, roix_huff_info* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    info->status = S->status;
    info->max_len = 0;
    info->n = n;
    info->n_blocks = (n + kHfBlock - 1) / kHfBlock;
    info->payload_words = 0ull;
    info->compressed_bytes = 0ull;
    info->pad[0] = info->pad[1] = info->pad[2] = 0ull;
}

// ------------------------------------------------------------ launchers

static size_t hf_align(size_t x) { return (x + 255) & ~(size_t)255; }

// the state, then the encoder's scan chunk sums or the decoder's three-code table
size_t huff_scratch_bytes() {
    const size_t scan = hf_align((size_t)(kScanBlocks + 1) * 8), tab3 = hf_align((size_t)(1 << kHf3Peek) * 4);
    return hf_align(sizeof(HfState)) + (scan > tab3 ? scan : tab3);
}




hipError_t launch_huff_encode(const LaunchCtx& lc, const uint8_t* in, int64_t n, uint8_t* lengths,
                              unsigned long long* block_off, uint16_t* sub_bits, uint32_t* payload, int64_t cap_words,
                              void* scratch, roix_huff_info* info) {
    HfState* S = (HfState*)scratch;
    uint64_t* tmp = (uint64_t*)((uint8_t*)scratch + hf_align(sizeof(HfState)));
    const unsigned long long N = (unsigned long long)n;
    const int64_t nb = (n + kHfBlock - 1) / kHfBlock;
    timer_begin(lc.timer, ST_HUFF, lc.stream);
    hipLaunchKernelGGL(k_hf_clear, dim3(1), dim3(256), 0, lc.stream, S);
    const int64_t hv = n / 16 / 256 + 1;
    const int hgrid = (int)(hv < (int64_t)lc.grid_stream ? hv : (int64_t)lc.grid_stream);
    hipLaunchKernelGGL(k_hf_hist, dim3(hgrid), dim3(256), 0, lc.stream, in, N, S);
    hipLaunchKernelGGL(k_hf_build, dim3(1), dim3(256), 0, lc.stream, S, lengths);
    const int bgrid = (int)(nb < 1 ? 1 : nb < (int64_t)lc.grid_stream * 4 ? nb : (int64_t)lc.grid_stream * 4);
    if (nb > 0) {
        hipLaunchKernelGGL(k_hf_count, dim3(bgrid), dim3(kWave), 0, lc.stream, in, N, (const HfState*)S,
                           block_off, sub_bits);
        hipError_t e = launch_scan_u64(lc, (const uint64_t*)block_off, (uint64_t*)block_off, nb,
                                       block_off + nb, tmp);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hf_encode, dim3(bgrid), dim3(kWave), 0, lc.stream, in, N, (const HfState*)S,
                           (const unsigned long long*)block_off, payload, (unsigned long long)cap_words);
    } else {
        hipLaunchKernelGGL(k_hf_zero_off, dim3(1), dim3(1), 0, lc.stream, block_off);
    }
    hipLaunchKernelGGL(k_hf_finalize, dim3(1), dim3(1), 0, lc.stream, (const HfState*)S,
                       (const unsigned long long*)block_off, N, (unsigned long long)cap_words, sub_bits ? 1 : 0,
                       info);
    timer_end(lc.timer, ST_HUFF, lc.stream);
    return hipGetLastError();
}

hipError_t launch_huff_decode(const LaunchCtx& lc, const uint8_t* lengths, const unsigned long long* block_off,
                              const uint16_t* sub_bits, const uint32_t* payload, int64_t payload_words, int64_t n,
                              uint8_t* out, void* scratch, roix_huff_info* info) {
    HfState* S = (HfState*)scratch;
    const unsigned long long N = (unsigned long long)n;
    const int64_t nb = (n + kHfBlock - 1) / kHfBlock;
    timer_begin(lc.timer, ST_HUFF, lc.stream);
    hipLaunchKernelGGL(k_hf_clear, dim3(1), dim3(256), 0, lc.stream, S);
    if (nb > 0) {
        const int64_t tasks = sub_bits ? nb * kHfSubs : nb;
        const int64_t g = (tasks + 255) / 256;
        const int grid = (int)(g < (int64_t)lc.grid_stream ? g : (int64_t)lc.grid_stream);
        const int vec = ((uintptr_t)payload & 15u) == 0u ? 1 : 0;
        if (sub_bits) {
            uint32_t* tab3 = (uint32_t*)((uint8_t*)scratch + hf_align(sizeof(HfState)));
            hipLaunchKernelGGL(k_hf_peek3, dim3((1 << kHf3Peek) / 256), dim3(256), 0, lc.stream, lengths, N, tab3, S);
            hipLaunchKernelGGL((k_hf_decode<true, true>), dim3(grid), dim3(256), 0, lc.stream, lengths, block_off,
                               sub_bits, payload, (unsigned long long)payload_words, N, out, S, vec,
                               (const uint32_t*)tab3);
        } else {
            hipLaunchKernelGGL((k_hf_decode<false, false>), dim3(grid), dim3(256), 0, lc.stream, lengths, block_off,
                               sub_bits, payload, (unsigned long long)payload_words, N, out, S, vec,
                               (const uint32_t*)nullptr);
        }
    }
    hipLaunchKernelGGL(k_hf_decode_finalize, dim3(1), dim3(1), 0, lc.stream, (const HfState*)S, N, info);
    timer_end(lc.timer, ST_HUFF, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
