/*
 * sanitize_driver.c - runs every entry point of the CPU oracle on small
 * inputs, for a build of the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (TEST INFRASTRUCTURE; the test suite compiles
 * and runs it).  It checks no values: the pins do that.  It exists so that an
 * out-of-bounds access, a leak or undefined arithmetic anywhere in the oracle
 * stops the run with the sanitizer's report.
 *
 * The oracle is included as one translation unit, so the driver sees its
 * types and static helpers exactly as compiled.
 */
#include "roix_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

/* xorshift64*: small, deterministic inputs for the driver only */
static uint64_t rnd(void) {
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}
static double urand(void) { return (double)(rnd() >> 11) * (1.0 / 9007199254740992.0); }

static int failures = 0;
#define EXPECT(c)                                                   \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "expectation failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                             \
        }                                                           \
    } while (0)

/* a volume of background noise with a few boxes and noisy voxels */
static void make_volume(float* f, uint16_t* u, int64_t nx, int64_t ny, int64_t nz) {
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t v = (z * ny + y) * nx + x;
                double val = 0.1 + 0.02 * (urand() - 0.5);
                if (x > nx / 4 && x < nx / 2 && y > 1 && y < ny - 2 && z > 0) val = 0.7 + 0.02 * urand();
                if (x > nx - 4 && y < 3) val = 0.8;
                if (urand() < 0.01) val = 0.9;
                if (f) f[v] = (float)val;
                if (u) u[v] = (uint16_t)(val * 60000.0);
            }
}

static void run_fused(const void* in, int dtype, int64_t nx, int64_t ny, int64_t nz, int eb_mode, double eb,
                      int thr, double fixed, int conn, int keep, int64_t min_size, int64_t rows_cap,
                      int64_t stream_cap, int64_t outl_cap, int64_t comps_cap, int decode) {
    const uint64_t N = (uint64_t)(nx * ny * nz);
    or_comp* comps = calloc((size_t)(comps_cap > 0 ? comps_cap : 1), sizeof(or_comp));
    or_row* rows = calloc((size_t)(rows_cap > 0 ? rows_cap : 1), sizeof(or_row));
    uint8_t* stream = calloc((size_t)(stream_cap > 0 ? stream_cap : 1), 1);
    float* outl = calloc((size_t)(outl_cap > 0 ? outl_cap : 1), sizeof(float));
    int32_t* slice = calloc((size_t)nz, sizeof(int32_t));
    or_fused_info info;
    const int st = oracle_fused(in, dtype, nx, ny, nz, eb_mode, eb, thr, fixed, conn, keep, min_size, comps,
                                comps_cap, rows, rows_cap, stream, stream_cap, outl, outl_cap, &info, slice);
    EXPECT(st >= 0 && st <= OR_ETRUNC);
    if (decode && st == OR_OK) {
        float* out = malloc(N * sizeof(float));
        const int d = oracle_decode(rows, info.n_rows, stream, outl, info.n_outliers, &info.q, nx, ny, nz, 0.0f,
                                    out);
        EXPECT(d == OR_OK);
        /* a corrupted table is refused, not read out of bounds */
        if (info.n_rows > 0) {
            rows[0].xe = (uint32_t)nx + 5u;
            EXPECT(oracle_decode(rows, info.n_rows, stream, outl, info.n_outliers, &info.q, nx, ny, nz, 0.0f,
                                 out) == OR_EINVAL);
        }
        free(out);
    }
    free(comps);
    free(rows);
    free(stream);
    free(outl);
    free(slice);
}

static void fused_cases(void) {
    const int64_t shapes[][3] = {{1, 1, 1}, {7, 5, 3}, {16, 12, 10}, {33, 9, 4}, {65, 3, 2}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
        const uint64_t N = (uint64_t)(nx * ny * nz);
        float* f = malloc(N * sizeof(float));
        uint16_t* u = malloc(N * sizeof(uint16_t));
        make_volume(f, u, nx, ny, nz);
        int64_t rc = ny * nz, sc = (int64_t)N * 4, oc = (int64_t)N, cc = (int64_t)N;
        for (int conn = 6; conn <= 26; conn += 20)
            for (int thr = OR_THR_OTSU; thr <= OR_THR_SLICE; ++thr)
                for (int keep = 0; keep < 2; ++keep) {
                    run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-3, thr, 0.5, conn, keep, 3, rc, sc, oc, cc, 1);
                    run_fused(u, OR_U16, nx, ny, nz, OR_EB_REL, 1e-4, thr, 30000.0, conn, keep, 1, rc, sc, oc, cc,
                              1);
                }
        /* tiny bound (escapes, 32-bit codes) and truncated outputs */
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-7, OR_THR_OTSU, 0.0, 26, 1, 1, rc, sc, oc, cc, 1);
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-3, OR_THR_OTSU, 0.0, 26, 1, 1, 1, 2, 0, 1, 0);
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-3, OR_THR_FIXED, 0.05, 6, 0, 1, 0, 0, 0, 0, 0);
        /* non-finite input, a bound that overflows the codes */
        f[N / 2] = NAN;
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-3, OR_THR_OTSU, 0.0, 26, 1, 1, rc, sc, oc, cc, 0);
        f[N / 2] = 1e30f;
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-9, OR_THR_OTSU, 0.0, 26, 1, 1, rc, sc, oc, cc, 0);
        /* constant volume with a relative bound */
        for (uint64_t v = 0; v < N; ++v) f[v] = 0.25f;
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_REL, 1e-3, OR_THR_OTSU, 0.0, 6, 1, 1, rc, sc, oc, cc, 0);
        run_fused(f, OR_F32, nx, ny, nz, OR_EB_ABS, 1e-3, OR_THR_MULTI4, 0.0, 6, 1, 1, rc, sc, oc, cc, 1);
        /* background subtraction and its reverse */
        float* bg = malloc((size_t)(nx * ny) * sizeof(float));
        float* m = malloc(N * sizeof(float));
        for (int64_t i = 0; i < nx * ny; ++i) bg[i] = (float)(0.01 * urand());
        EXPECT(oracle_background(u, OR_U16, bg, 1, nx, ny, nz, 0, m) == OR_OK);
        EXPECT(oracle_background(m, OR_F32, bg, 1, nx, ny, nz, 1, m) == OR_OK);
        EXPECT(oracle_background(m, OR_F32, bg, 2 + nz, nx, ny, nz, 0, m) == OR_EINVAL);
        free(bg);
        free(m);
        free(f);
        free(u);
    }
}

static void abs_quantize_cases(void) {
    const uint64_t sizes[] = {0, 1, 2, 255, 256, 257, 4099};
    const double tols[] = {0.0, 0.4, 1.0, 1.5, 3.0, 127.0, 300.0, 5000.0};
    for (size_t a = 0; a < sizeof sizes / sizeof sizes[0]; ++a)
        for (size_t b = 0; b < sizeof tols / sizeof tols[0]; ++b) {
            const uint64_t m = sizes[a];
            uint8_t* d = malloc(m ? m : 1);
            uint8_t* q = malloc(m ? m : 1);
            for (uint64_t i = 0; i < m; ++i) d[i] = (uint8_t)(i % 3 == 0 ? rnd() : (i * 7) & 255);
            uint64_t groups = 0;
            EXPECT(oracle_abs_quantize(d, m, tols[b], q, &groups) == OR_OK);
            EXPECT(groups <= m);
            free(d);
            free(q);
        }
    uint64_t g = 0;
    uint8_t one = 5, out = 0;
    EXPECT(oracle_abs_quantize(&one, 1, -1.0, &out, &g) == OR_EINVAL);
    EXPECT(oracle_abs_quantize(&one, 1, NAN, &out, &g) == OR_EINVAL);
}

static void huffman_cases(void) {
    const uint64_t sizes[] = {0, 1, 4095, 4096, 4097, 9000};
    for (size_t a = 0; a < sizeof sizes / sizeof sizes[0]; ++a)
        for (int kind = 0; kind < 3; ++kind) {
            const uint64_t n = sizes[a];
            uint8_t* in = malloc(n ? n : 1);
            for (uint64_t i = 0; i < n; ++i)
                in[i] = kind == 0 ? 7 : kind == 1 ? (uint8_t)rnd() : (uint8_t)(rnd() % 97 < 90 ? 0 : rnd() % 5);
            const uint64_t nb = (n + OR_HUFF_BLOCK - 1) / OR_HUFF_BLOCK;
            uint8_t len[256];
            uint64_t* off = calloc(nb + 1, sizeof(uint64_t));
            const uint64_t cap = n / 4 * 9 + 16;
            uint32_t* payload = calloc(cap, sizeof(uint32_t));
            uint64_t words = 0;
            uint16_t* sub = calloc(nb * OR_HUFF_SUBS + 1, sizeof(uint16_t));
            int st = oracle_huff_encode(in, n, len, off, payload, cap, &words, sub);
            EXPECT(st == OR_OK || (n == 0 && st != OR_OK));
            if (st == OR_OK) {
                uint8_t* back = malloc(n ? n : 1);
                EXPECT(oracle_huff_decode(len, off, payload, words, n, back, NULL) == OR_OK);
                EXPECT(n == 0 || memcmp(back, in, n) == 0);
                EXPECT(oracle_huff_decode(len, off, payload, words, n, back, sub) == OR_OK);
                EXPECT(n == 0 || memcmp(back, in, n) == 0);
                /* a payload cut short is refused, not read past its end */
                if (words > 0) EXPECT(oracle_huff_decode(len, off, payload, words - 1, n, back, NULL) == OR_EINVAL);
                if (words > 0) EXPECT(oracle_huff_decode(len, off, payload, words - 1, n, back, sub) == OR_EINVAL);
                /* a sub-block length one bit off is refused */
                if (nb > 0) {
                    sub[0] += 1;
                    EXPECT(oracle_huff_decode(len, off, payload, words, n, back, sub) == OR_EINVAL);
                    sub[0] -= 1;
                }
                free(back);
                /* a truncated capacity reports the size it needed */
                uint64_t w2 = 0;
                if (words > 0) EXPECT(oracle_huff_encode(in, n, len, off, payload, words - 1, &w2, NULL) == OR_ETRUNC);
            }
            free(in);
            free(off);
            free(payload);
            free(sub);
        }
}

int main(void) {
    fused_cases();
    abs_quantize_cases();
    huffman_cases();
    int64_t sizes[8] = {0};
    oracle_sizes(sizes);
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
