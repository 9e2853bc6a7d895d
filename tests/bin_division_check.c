/* Exhaustive check of the two exact integer forms of the histogram bin
 * floor(256 u / K) that the HIP kernels use instead of a division:
 *   fast:  M = ceil(2^40 / K), bin = (u * M) >> 32        for K <= 65536
 *   24-bit: the smallest a with m = ceil(2^(40-a) / K) < 2^24, usable when
 *          K^2 2^a <= 2^32 and (K - 1) 2^a < 2^24; bin = ((u << a) * m) >> 32
 * for every K and every u < K.  Prints the largest K with a 24-bit form and
 * exits non-zero on any mismatch. */
#include <stdint.h>
#include <stdio.h>

static int pick24(uint64_t K, unsigned* a_out, uint64_t* m_out) {
    for (unsigned a = 0; a <= 24; ++a) {
        const uint64_t m = ((1ull << (40 - a)) + K - 1) / K;
        if (m >= (1ull << 24)) continue;
        if (K * K * (1ull << a) > (1ull << 32) || ((K - 1) << a) >= (1ull << 24)) return 0;
        *a_out = a;
        *m_out = m;
        return 1;
    }
    return 0;
}

int main(void) {
    uint64_t bad = 0, max24 = 0;
    for (uint64_t K = 1; K <= 65536; ++K) {
        const uint64_t M = ((1ull << 40) + K - 1) / K;
        unsigned a = 0;
        uint64_t m = 0;
        const int has24 = pick24(K, &a, &m);
        if (has24) max24 = K;
        for (uint64_t u = 0; u < K; ++u) {
            const uint64_t want = (256 * u) / K;
            if (((u * M) >> 32) != want) ++bad;
            if (has24 && ((((u << a) & 0xFFFFFFull) * m) >> 32) != want) ++bad;
        }
    }
    printf("max_k24 %llu bad %llu\n", (unsigned long long)max24, (unsigned long long)bad);
    return bad ? 1 : 0;
}
