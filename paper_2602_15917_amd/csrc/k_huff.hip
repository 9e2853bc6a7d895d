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
// count (for an
// exclusive scan of the block sizes), and the codes, ORed into the block's
// words in LDS at the positions a wave prefix sum gives, then copied out.
// Decoding: a lane per block with a 64-bit bit window, a 10-bit lookup table
// and a canonical search for longer codes.
#include "common.h"

namespace roix {

constexpr int kHfBlock = 4096;   // input bytes per block
constexpr int kHfPeek = 10;      // bits of the decoder's lookup table

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
    __shared__ int ns_sh;
    __shared__ uint32_t bl_count[34], next_code[34];
    __shared__ unsigned long long hs[256];
    __shared__ uint8_t lens[256];
    __shared__ uint32_t codes[256];
    const int t = threadIdx.x;
    const unsigned long long c = S->hist[t];
    hs[t] = c;
    // rank of this byte among the used ones by (count, byte value)
    if (t == 0) ns_sh = 0;
    __syncthreads();
    if (c) atomicAdd(&ns_sh, 1);
    int rank = 0;
    for (int u = 0; u < 256; ++u) {
        const unsigned long long cu = hs[u];
        rank += (cu && (cu < c || (cu == c && u < t))) ? 1 : 0;
    }
    __syncthreads();
    if (c) sym[rank] = t;
    lens[t] = 0;
    __syncthreads();
    const int ns = ns_sh;
    if (t == 0) {
        int maxl = 0;
        bool ok = true;
        if (ns == 1) {
            lens[sym[0]] = 1;
            maxl = 1;
        } else if (ns > 1) {
            for (int i = 0; i < ns; ++i) w[i] = hs[sym[i]];
            int lq = 0, mq = ns, next = ns;
            while (next < 2 * ns - 1) {
                int pick[2];
                for (int k = 0; k < 2; ++k) {
                    if (lq < ns && (mq >= next || w[lq] <= w[mq])) pick[k] = lq++;
                    else pick[k] = mq++;
                }
                w[next] = w[pick[0]] + w[pick[1]];
                parent[pick[0]] = next;
                parent[pick[1]] = next;
                ++next;
            }
            // depths, the root first (stored over the weights, no longer needed)
            int* depth = reinterpret_cast<int*>(w);
            depth[2 * ns - 2] = 0;
            for (int i = 2 * ns - 3; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
            for (int i = 0; i < ns; ++i) {
                const int d = depth[i];
                maxl = d > maxl ? d : maxl;
                if (d > 32) ok = false;
                lens[sym[i]] = (uint8_t)(d > 32 ? 0 : d);
            }
        }
        S->max_len = maxl;
        if (!ok) S->status = ROIX_ERANGE;
        // canonical codes
        for (int i = 0; i < 34; ++i) bl_count[i] = next_code[i] = 0u;
        for (int i = 0; i < 256; ++i) bl_count[lens[i]]++;
        bl_count[0] = 0u;
        unsigned long long cc = 0ull;
        for (int b = 1; b <= 32; ++b) {
            cc = (cc + bl_count[b - 1]) << 1;
            next_code[b] = (uint32_t)cc;
        }
        for (int i = 0; i < 256; ++i) codes[i] = lens[i] ? next_code[lens[i]]++ : 0u;
    }
    __syncthreads();
    S->len[t] = lens[t];
    S->code[t] = codes[t];
    if (lengths_out) lengths_out[t] = lens[t];
}

// ------------------------------------------------------------ encoding

// bits of the 64 bytes lane `lane` holds of block b (len from LDS)
__device__ __forceinline__ uint32_t hf_lane_bits(const uint8_t* in, unsigned long long n, unsigned long long b, int lane,
                                                 const uint8_t* len, uint4* v) {
    const unsigned long long p0 = b * kHfBlock + 64ull * lane;
    uint32_t bits = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const unsigned long long p = p0 + 16ull * i;
        if (p + 16 <= n) {
            v[i] = ld_stream(reinterpret_cast<const uint4*>(in + p));
        } else {
            uint32_t ww[4] = {0u, 0u, 0u, 0u};
            for (int k = 0; k < 16; ++k)
                if (p + k < n) ww[k >> 2] |= (uint32_t)in[p + k] << (8 * (k & 3));
            v[i] = make_uint4(ww[0], ww[1], ww[2], ww[3]);
        }
    }
    const int cnt = p0 >= n ? 0 : (n - p0 >= 64 ? 64 : (int)(n - p0));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t ww[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (16 * i + k < cnt) bits += len[(ww[k >> 2] >> (8 * (k & 3))) & 0xFFu];
    }
    return bits;
}

__global__ __launch_bounds__(kWave) void k_hf_count(const uint8_t* __restrict__ in, unsigned long long n,
                                                    const HfState* S, unsigned long long* block_words) {
    __shared__ uint8_t len[256];
    for (int i = threadIdx.x; i < 256; i += kWave) len[i] = S->len[i];
    __syncthreads();
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    for (unsigned long long b = blockIdx.x; b < nb; b += gridDim.x) {
        uint4 v[4];
        const uint32_t bits = wave_sum(hf_lane_bits(in, n, b, threadIdx.x, len, v));
        if (threadIdx.x == 0) block_words[b] = (bits + 31u) / 32u;
    }
}

__global__ __launch_bounds__(kWave) void k_hf_encode(const uint8_t* __restrict__ in, unsigned long long n,
                                                     const HfState* S, const unsigned long long* block_off,
                                                     uint32_t* __restrict__ payload, unsigned long long cap_words) {
    __shared__ uint8_t len[256];
    __shared__ uint32_t code[256];
    __shared__ uint32_t buf[kHfBlock];  // a block's words: 32 bits per byte at most
    const int lane = threadIdx.x;
    for (int i = lane; i < 256; i += kWave) {
        len[i] = S->len[i];
        code[i] = S->code[i];
    }
    __syncthreads();
    if (S->status != 0) return;
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    for (unsigned long long b = blockIdx.x; b < nb; b += gridDim.x) {
        const unsigned long long w0 = block_off[b], w1 = block_off[b + 1];
        if (w1 > cap_words) continue;  // the payload does not hold this block (reported as ETRUNC)
        const uint32_t words = (uint32_t)(w1 - w0);
        __syncthreads();
        for (uint32_t i = lane; i < words; i += kWave) buf[i] = 0u;
        uint4 v[4];
        const uint32_t bits = hf_lane_bits(in, n, b, lane, len, v);
        // exclusive prefix of the lanes' bit counts
        uint32_t pos = bits;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t u = __shfl_up(pos, o);
            if (lane >= o) pos += u;
        }
        pos -= bits;
        __syncthreads();
        const unsigned long long p0 = b * kHfBlock + 64ull * lane;
        const int cnt = p0 >= n ? 0 : (n - p0 >= 64 ? 64 : (int)(n - p0));
        // the lane's bits [pos, pos + bits) gather in a 64-bit accumulator
        // (acc_n bits, most significant first); whole words go out with
        // plain stores except the lane's first and last, which neighbours
        // may share (ORed)
        const uint32_t first_w = pos >> 5, last_w = (pos + bits - 1u) >> 5;
        unsigned long long acc = 0ull;
        uint32_t acc_n = pos & 31u;  // the word starts before the lane's first bit: zeros there
        uint32_t wi = first_w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t ww[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (16 * i + k < cnt) {
                    const uint32_t sy = (ww[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                    const uint32_t L = len[sy];
                    acc |= (unsigned long long)code[sy] << (64u - acc_n - L);
                    acc_n += L;
                    if (acc_n >= 32u) {
                        const uint32_t word = (uint32_t)(acc >> 32);
                        if (wi == first_w || wi == last_w) atomicOr(&buf[wi], word);
                        else buf[wi] = word;
                        ++wi;
                        acc <<= 32;
                        acc_n -= 32u;
                    }
                }
            }
        }
        if (bits > 0u && acc_n > 0u) atomicOr(&buf[wi], (uint32_t)(acc >> 32));
        __syncthreads();
        for (uint32_t i = lane; i < words; i += kWave) payload[w0 + i] = buf[i];
    }
}

__global__ void k_hf_zero_off(unsigned long long* block_off) { block_off[0] = 0ull; }

__global__ void k_hf_finalize(const HfState* S, const unsigned long long* block_off, unsigned long long n,
                              unsigned long long cap_words, roix_huff_info* info) {
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
    info->compressed_bytes = 256ull + 8ull * (nb + 1) + 4ull * words;
    info->pad[0] = info->pad[1] = info->pad[2] = 0ull;
}

// ------------------------------------------------------------ decoding

struct HfDecode {
    uint32_t first[34];   // first canonical code of each length
    uint32_t count[34];   // codes of each length
    uint32_t index[34];   // position of a length's first byte in sym
    uint8_t sym[256];     // bytes by (length, value)
    uint16_t peek[1 << kHfPeek];  // top bits -> len << 8 | byte (len 0: longer code)
};

__global__ __launch_bounds__(256) void k_hf_decode(const uint8_t* lengths, const unsigned long long* block_off,
                                                   const uint32_t* payload, unsigned long long payload_words,
                                                   unsigned long long n, uint8_t* out, HfState* S) {
    __shared__ HfDecode T;
    __shared__ int bad_table;
    __shared__ uint32_t fill[34];
    const int t = threadIdx.x;
    if (t == 0) {
        bad_table = 0;
        for (int i = 0; i < 34; ++i) T.count[i] = 0u;
        unsigned long long kraft = 0ull;  // in units of 2^-32
        int used = 0;
        for (int i = 0; i < 256; ++i) {
            const int L = lengths[i];
            if (L > 32) bad_table = 1;
            else if (L) {
                T.count[L]++;
                kraft += 1ull << (32 - L);
                ++used;
            }
        }
        if (kraft > (1ull << 32) || (n > 0 && used == 0)) bad_table = 1;
        uint32_t pos = 0u;
        unsigned long long c = 0ull;
        for (int L = 1; L <= 32; ++L) {
            c = (c + (L > 1 ? T.count[L - 1] : 0u)) << 1;
            T.first[L] = (uint32_t)c;
            T.index[L] = pos;
            pos += T.count[L];
        }
        fill[0] = 0u;
        for (int L = 1; L <= 32; ++L) fill[L] = T.index[L];
        for (int i = 0; i < 256; ++i)
            if (lengths[i] && lengths[i] <= 32) T.sym[fill[lengths[i]]++] = (uint8_t)i;
    }
    __syncthreads();
    for (int e = t; e < (1 << kHfPeek); e += blockDim.x) {
        uint16_t val = 0;
        for (int L = 1; L <= kHfPeek && val == 0; ++L) {
            const uint32_t c = (uint32_t)e >> (kHfPeek - L);
            if (T.count[L] && c - T.first[L] < T.count[L])
                val = (uint16_t)((L << 8) | T.sym[T.index[L] + (c - T.first[L])]);
        }
        T.peek[e] = val;
    }
    __syncthreads();
    if (bad_table) {
        if (t == 0) atomicCAS(&S->status, 0, ROIX_EINVAL);
        return;
    }
    const unsigned long long nb = (n + kHfBlock - 1) / kHfBlock;
    for (unsigned long long b = (unsigned long long)blockIdx.x * blockDim.x + t; b < nb;
         b += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long w0 = block_off[b], w1 = block_off[b + 1];
        if ((b == 0 && w0 != 0) || w1 < w0 || w1 > payload_words) {
            atomicCAS(&S->status, 0, ROIX_EINVAL);
            continue;
        }
        const unsigned long long e = (b + 1) * kHfBlock < n ? (b + 1) * kHfBlock : n;
        unsigned long long wp = w0;          // next payload word to read
        unsigned long long window = 0ull;    // bits, the next one most significant
        int have = 0;
        bool ok = true;
        uint32_t acc = 0u;
        for (unsigned long long i = b * kHfBlock; i < e; ++i) {
            if (have <= 32 && wp < w1) {
                window |= (unsigned long long)payload[wp++] << (32 - have);
                have += 32;
            }
            const uint16_t pk = T.peek[window >> (64 - kHfPeek)];
            int L = pk >> 8;
            uint32_t s = pk & 0xFFu;
            if (L == 0) {  // a code longer than the table
                for (L = kHfPeek + 1; L <= 32; ++L) {
                    const uint32_t c = (uint32_t)(window >> (64 - L));
                    if (T.count[L] && c - T.first[L] < T.count[L]) {
                        s = T.sym[T.index[L] + (c - T.first[L])];
                        break;
                    }
                }
            }
            if (L > 32 || L > have) {
                ok = false;
                break;
            }
            window <<= L;
            have -= L;
            acc |= s << (8 * (i & 3));
            if ((i & 3) == 3 || i + 1 == e) {
                const unsigned long long a = i & ~3ull;
                if (a + 4 <= n) {
                    *reinterpret_cast<uint32_t*>(out + a) = acc;
                } else {
                    for (unsigned long long k = a; k < n; ++k) out[k] = (uint8_t)(acc >> (8 * (k - a)));
                }
                acc = 0u;
            }
        }
        if (!ok) atomicCAS(&S->status, 0, ROIX_EINVAL);
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

size_t huff_scratch_bytes() { return hf_align(sizeof(HfState)) + hf_align((size_t)(kScanBlocks + 1) * 8); }

hipError_t launch_huff_encode(const LaunchCtx& lc, const uint8_t* in, int64_t n, uint8_t* lengths,
                              unsigned long long* block_off, uint32_t* payload, int64_t cap_words, void* scratch,
                              roix_huff_info* info) {
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
                           block_off);
        hipError_t e = launch_scan_u64(lc, (const uint64_t*)block_off, (uint64_t*)block_off, nb,
                                       block_off + nb, tmp);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hf_encode, dim3(bgrid), dim3(kWave), 0, lc.stream, in, N, (const HfState*)S,
                           (const unsigned long long*)block_off, payload, (unsigned long long)cap_words);
    } else {
        hipLaunchKernelGGL(k_hf_zero_off, dim3(1), dim3(1), 0, lc.stream, block_off);
    }
    hipLaunchKernelGGL(k_hf_finalize, dim3(1), dim3(1), 0, lc.stream, (const HfState*)S,
                       (const unsigned long long*)block_off, N, (unsigned long long)cap_words, info);
    timer_end(lc.timer, ST_HUFF, lc.stream);
    return hipGetLastError();
}

hipError_t launch_huff_decode(const LaunchCtx& lc, const uint8_t* lengths, const unsigned long long* block_off,
                              const uint32_t* payload, int64_t payload_words, int64_t n, uint8_t* out,
                              void* scratch, roix_huff_info* info) {
    HfState* S = (HfState*)scratch;
    const unsigned long long N = (unsigned long long)n;
    const int64_t nb = (n + kHfBlock - 1) / kHfBlock;
    timer_begin(lc.timer, ST_HUFF, lc.stream);
    hipLaunchKernelGGL(k_hf_clear, dim3(1), dim3(256), 0, lc.stream, S);
    if (nb > 0) {
        const int64_t g = (nb + 255) / 256;
        const int grid = (int)(g < (int64_t)lc.grid_stream ? g : (int64_t)lc.grid_stream);
        hipLaunchKernelGGL(k_hf_decode, dim3(grid), dim3(256), 0, lc.stream, lengths, block_off, payload,
                           (unsigned long long)payload_words, N, out, S);
    }
    hipLaunchKernelGGL(k_hf_decode_finalize, dim3(1), dim3(1), 0, lc.stream, (const HfState*)S, N, info);
    timer_end(lc.timer, ST_HUFF, lc.stream);
    return hipGetLastError();
}

}  // namespace roix
