/*
 * roix_oracle.c - CPU oracle for the ROI reduction path (TEST INFRASTRUCTURE).
 *
 * This is the plain, slow, single-threaded reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it; the GPU library never links, includes or calls
 * it, and it shares no code, header or table with the GPU sources.
 *
 * Build: gcc -O2 -ffp-contract=off (no -ffast-math, no -march=native), so
 * every float operation below is one IEEE-754 binary32/binary64 operation in
 * round-to-nearest-even, with no fused multiply-add.
 *
 * What it computes (ROIX-Comp, arXiv 2602.15917), step by step:
 *   range        I_max of the normalisation (Sec. 4.1.2, Eq. 1) and the value
 *                range a relative error bound refers to
 *   resolve      the positive absolute tolerance E_abs of the quantiser's
 *                problem statement (Sec. 4.2.3), as an fp32 bound
 *   quantise     per-voxel code q with |x - q*2eb| <= eb, or an escape
 *                (outlier) when fp32 rounding would break the bound
 *                (Sec. 4.2.3 problem statement; a per-voxel fp32 formula
 *                takes the place of the paper's sequential grouping)
 *   histogram    256 equal bins over the code range: the 8-bit normalisation
 *                of Sec. 4.1.2 applied to codes
 *   threshold    two-class Otsu (1979) on those bins (Sec. 4.1.3), the
 *                multi-level Otsu of Liao, Chen & Chung (2001) that Sec.
 *                4.1.3 names (3 or 4 classes; object = above the lowest
 *                threshold), or a fixed threshold; pixels above the
 *                threshold are object
 *   binarise     mask M = 1 for object voxels (Sec. 4.1.4, Eq. 2)
 *   label        connected components of the mask in 3-D (6 or 26
 *                neighbours): the volumetric form of the outer-contour
 *                detection of Sec. 4.2.1; label = smallest linear index
 *   keep         the largest component by voxel count (Sec. 4.2.1), or every
 *                component of at least min_size voxels
 *   rows         per row (z,y) the leftmost and rightmost kept voxel:
 *                G(i) = [i, x_start, x_end] (Sec. 4.2.2, Eq. 3), half-open
 *   stream       the pixel section P(i) (Sec. 4.2.2, Eq. 4) as codes of
 *                b bits, with the raw value of every outlier kept aside
 *   decode       the reverse process of Sec. 4.3 (rows restored from the
 *                geometry section)
 *   background   background subtraction M = I - B of Sec. 4.1.1 (B a
 *                calibration plane or volume), and M + B to put a decoded
 *                volume back on its background
 *   section      the normalised 8-bit pixel section of the extraction (Sec.
 *                4.1.2, Eq. 1): the histogram level of every span voxel's code
 *   abs_quantize the paper's own absolute error-bounded quantisation of an
 *                8-bit pixel sequence (Sec. 4.2.3): the longest runs whose
 *                largest and smallest pixel differ by at most 2E, each
 *                written as floor((min + max) / 2)
 *   huffman      a lossless entropy stage for the packed stream (the Huffman
 *                coding the paper lists among lossless coders, Sec. 1):
 *                byte counts, Huffman code lengths, canonical codes, the
 *                bytes coded in blocks of 4096, and the decoder
 *
 * Where the paper is silent or ambiguous this file takes these readings:
 * half-open spans [x_start, x_end) so that n_i = x_end - x_start; a span
 * covers every voxel between the extreme kept voxels of its row; two-class
 * Otsu with the first maximum winning ties; "above the threshold" is strict;
 * LARGEST ties go to the smallest label; 8-bit bins span [qmin, qmax].
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { OR_OK = 0, OR_EINVAL = 1, OR_ERANGE = 2, OR_ENOMEM = 3, OR_ETRUNC = 4 };
enum { OR_F32 = 0, OR_U16 = 1 };
enum { OR_EB_ABS = 0, OR_EB_REL = 1 };
enum { OR_THR_OTSU = 0, OR_THR_FIXED = 1, OR_THR_MULTI3 = 2, OR_THR_MULTI4 = 3, OR_THR_SLICE = 4 };
enum { OR_KEEP_MIN_SIZE = 0, OR_KEEP_LARGEST = 1 };
enum { OR_FLAG_DEGENERATE = 1u, OR_FLAG_EMPTY_ROI = 2u, OR_FLAG_FIXED = 4u, OR_FLAG_SLICE = 8u };

typedef struct {
    int32_t status;
    float xmin, xmax, eb32, w, r;
    int32_t qmin, qmax;
    int64_t K;
    int32_t width_bits;
    uint32_t esc;
} or_params;

typedef struct {
    uint64_t label, size;
    uint32_t x0, x1, y0, y1, z0, z1; /* half-open bounding box */
    uint32_t kept, pad;
} or_comp;

typedef struct {
    uint32_t z, y, xs, xe; /* span [xs, xe) of row (z, y) */
    uint64_t code_off, outlier_off;
} or_row;

typedef struct {
    or_params q;
    int32_t seg_status, otsu_bin, q_thr;
    uint32_t flags;
    uint64_t hist[256];
    uint64_t n_mask, n_components, n_kept, n_kept_voxels;
    uint32_t bbox[6];
    int32_t ext_status, pad;
    uint64_t n_rows, n_codes, n_outliers, stream_bytes;
    double stage_seconds[8]; /* range+resolve, histogram, threshold+mask, label, keep, rows, stream, total */
    int32_t thresholds[3];   /* multi-level Otsu: t1 < t2 (< t3), -1 unused; two-class Otsu: t*; else -1 */
    int32_t n_classes;
} or_fused_info;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static float voxel(const void* in, int dtype, uint64_t v) {
    return dtype == OR_F32 ? ((const float*)in)[v] : (float)((const uint16_t*)in)[v];
}

/* ------------------------------------------------------------------ range */

/* a < b in the IEEE total order restricted to finite values (-0 < +0) */
static int total_less(float a, float b) {
    if (a < b) return 1;
    if (a > b) return 0;
    return signbit(a) && !signbit(b);
}

/* xmin, xmax over every voxel; a NaN or infinity is an invalid input. */
int oracle_range(const void* in, int dtype, uint64_t n, float* xmin, float* xmax) {
    if (n == 0) return OR_EINVAL;
    float lo = voxel(in, dtype, 0), hi = lo;
    for (uint64_t v = 0; v < n; ++v) {
        float x = voxel(in, dtype, v);
        if (!isfinite(x)) return OR_EINVAL;
        if (total_less(x, lo)) lo = x;
        if (total_less(hi, x)) hi = x;
    }
    *xmin = lo;
    *xmax = hi;
    return OR_OK;
}

/* ---------------------------------------------------------------- resolve */

/* The error bound: E_abs must be positive (Sec. 4.2.3).  A relative bound is
 * a fraction of the value range.  The fp32 bound is the largest float not
 * above the requested one, so |x - xhat| <= eb32 implies the f64 bound. */
int oracle_resolve(float xmin, float xmax, int eb_mode, double eb_value, or_params* p) {
    memset(p, 0, sizeof *p);
    p->xmin = xmin;
    p->xmax = xmax;
    double eb = eb_mode == OR_EB_ABS ? eb_value : eb_value * ((double)xmax - (double)xmin);
    if (!(eb > 0.0) || !isfinite(eb)) return p->status = OR_EINVAL;
    float eb32 = (float)eb;
    if ((double)eb32 > eb) eb32 = nextafterf(eb32, 0.0f);
    if (!isnormal(eb32)) return p->status = OR_EINVAL;
    float w = eb32 + eb32; /* bin width 2*eb: every x within eb of some q*w */
    float r = 1.0f / w;
    if (!isfinite(w) || !isfinite(r) || r == 0.0f) return p->status = OR_EINVAL;
    p->eb32 = eb32;
    p->w = w;
    p->r = r;
    float qlo = xmin * r, qhi = xmax * r;
    if (!(fabsf(qlo) <= 16777216.0f) || !(fabsf(qhi) <= 16777216.0f)) return p->status = OR_ERANGE;
    p->qmin = (int32_t)rintf(qlo);
    p->qmax = (int32_t)rintf(qhi);
    p->K = (int64_t)p->qmax - (int64_t)p->qmin + 1;
    p->width_bits = p->K <= 255 ? 8 : (p->K <= 65535 ? 16 : 32);
    p->esc = p->width_bits == 32 ? 0xFFFFFFFFu : ((1u << p->width_bits) - 1u);
    return p->status = OR_OK;
}

/* --------------------------------------------------------------- quantise */

/* code of one value: nearest multiple of w (ties to even), in fp32 */
static int32_t code_of(float x, const or_params* p) {
    float t = x * p->r;
    return (int32_t)rintf(t);
}

/* escape when fp32 rounding puts the reconstruction outside the bound */
static int is_outlier(float x, int32_t q, const or_params* p) {
    float xhat = (float)q * p->w;
    float d = x - xhat;
    return !(fabsf(d) <= p->eb32);
}

int oracle_quantize(const void* in, int dtype, uint64_t n, const or_params* p, int32_t* codes,
                    uint32_t* outlier_bits, uint64_t* n_outliers) {
    if (p->status != OR_OK) return p->status;
    uint64_t cnt = 0;
    if (outlier_bits) memset(outlier_bits, 0, sizeof(uint32_t) * (size_t)((n + 31) / 32));
    for (uint64_t v = 0; v < n; ++v) {
        float x = voxel(in, dtype, v);
        int32_t q = code_of(x, p);
        if (codes) codes[v] = q;
        if (is_outlier(x, q, p)) {
            ++cnt;
            if (outlier_bits) outlier_bits[v / 32] |= 1u << (v % 32);
        }
    }
    if (n_outliers) *n_outliers = cnt;
    return OR_OK;
}

/* -------------------------------------------------------------- histogram */

/* 8-bit normalisation of Eq. 1 applied to the code range [qmin, qmax]:
 * bin = floor(256 (q - qmin) / K), exact in integers. */
static int bin_of(int32_t q, const or_params* p) {
    int64_t u = (int64_t)q - (int64_t)p->qmin;
    return (int)((u * 256) / p->K);
}

void oracle_histogram_codes(const int32_t* codes, uint64_t n, const or_params* p, uint64_t hist[256]) {
    memset(hist, 0, sizeof(uint64_t) * 256);
    for (uint64_t v = 0; v < n; ++v) hist[bin_of(codes[v], p)]++;
}

/* ------------------------------------------------------------------- Otsu */

/* Otsu (1979): the split t maximising the between-class variance, evaluated
 * as W0*W1*(m0 - m1)^2 (same argmax as the variance, which divides by NT^2).
 * Class 0 holds bins 0..t, class 1 bins t+1..255.  Splits with an empty class
 * are skipped; the first maximum wins.  Returns flags; *t_star = 255 (empty
 * mask) when no split has two non-empty classes. */
uint32_t oracle_otsu(const uint64_t hist[256], int32_t* t_star) {
    uint64_t NT = 0, ST = 0;
    for (int i = 0; i < 256; ++i) {
        NT += hist[i];
        ST += (uint64_t)i * hist[i];
    }
    uint64_t W0 = 0, S0 = 0;
    double best = -1.0;
    int32_t t_best = 255;
    for (int t = 0; t < 255; ++t) {
        W0 += hist[t];
        S0 += (uint64_t)t * hist[t];
        uint64_t W1 = NT - W0;
        if (W0 == 0 || W1 == 0) continue;
        double m0 = (double)S0 / (double)W0;
        double m1 = (double)(ST - S0) / (double)W1;
        double d = m0 - m1;
        double s = (((double)W0 * (double)W1) * d) * d;
        if (s > best) {
            best = s;
            t_best = t;
        }
    }
    *t_star = t_best;
    return best < 0.0 ? OR_FLAG_DEGENERATE : 0u;
}

/* Multi-level Otsu (Liao, Chen & Chung 2001), K = 3 or 4 classes: the
 * thresholds t1 < .. < t_{K-1} in 0..254 maximising the between-class
 * variance.  For a fixed histogram that variance is (1/NT) sum_k S_k^2 / W_k
 * minus a constant (W_k voxels and S_k the bin sum of class k), so the
 * search maximises sum_k S_k^2 / W_k, evaluated in binary64 in class order:
 * ((S_0^2 / W_0 + S_1^2 / W_1) + S_2^2 / W_2) (+ S_3^2 / W_3).  Class k
 * holds bins t_k + 1 .. t_{k+1} (t_0 = -1, t_K = 255).  Tuples with an empty
 * class are skipped and the first maximum in lexicographic order of the
 * tuple wins.  t[] receives the thresholds (-1 for an unused slot); with no
 * valid tuple every threshold is 255 (empty mask).  Returns flags. */
static double class_term(uint64_t W, uint64_t S) {
    double s = (double)S;
    return (s * s) / (double)W;
}

uint32_t oracle_multi_otsu(const uint64_t hist[256], int classes, int32_t t[3]) {
    uint64_t P[257], Q[257]; /* P[i], Q[i]: voxels and bin sum of bins 0 .. i-1 */
    P[0] = Q[0] = 0;
    for (int i = 0; i < 256; ++i) {
        P[i + 1] = P[i] + hist[i];
        Q[i + 1] = Q[i] + (uint64_t)i * hist[i];
    }
    double best = -1.0;
    int32_t b1 = 255, b2 = 255, b3 = 255;
    if (classes == 3) {
        for (int t1 = 0; t1 < 254; ++t1)
            for (int t2 = t1 + 1; t2 < 255; ++t2) {
                uint64_t W0 = P[t1 + 1], W1 = P[t2 + 1] - P[t1 + 1], W2 = P[256] - P[t2 + 1];
                if (!W0 || !W1 || !W2) continue;
                uint64_t S0 = Q[t1 + 1], S1 = Q[t2 + 1] - Q[t1 + 1], S2 = Q[256] - Q[t2 + 1];
                double v = (class_term(W0, S0) + class_term(W1, S1)) + class_term(W2, S2);
                if (v > best) {
                    best = v;
                    b1 = t1;
                    b2 = t2;
                }
            }
        t[0] = b1;
        t[1] = b2;
        t[2] = -1;
    } else {
        for (int t1 = 0; t1 < 253; ++t1)
            for (int t2 = t1 + 1; t2 < 254; ++t2)
                for (int t3 = t2 + 1; t3 < 255; ++t3) {
                    uint64_t W0 = P[t1 + 1], W1 = P[t2 + 1] - P[t1 + 1], W2 = P[t3 + 1] - P[t2 + 1],
                             W3 = P[256] - P[t3 + 1];
                    if (!W0 || !W1 || !W2 || !W3) continue;
                    uint64_t S0 = Q[t1 + 1], S1 = Q[t2 + 1] - Q[t1 + 1], S2 = Q[t3 + 1] - Q[t2 + 1],
                             S3 = Q[256] - Q[t3 + 1];
                    double v = ((class_term(W0, S0) + class_term(W1, S1)) + class_term(W2, S2)) + class_term(W3, S3);
                    if (v > best) {
                        best = v;
                        b1 = t1;
                        b2 = t2;
                        b3 = t3;
                    }
                }
        t[0] = b1;
        t[1] = b2;
        t[2] = b3;
    }
    return best < 0.0 ? OR_FLAG_DEGENERATE : 0u;
}

/* smallest code in the object class.  Otsu: bins above t*, i.e.
 * floor(256 u / K) >= t*+1  <=>  u >= ceil((t*+1) K / 256).
 * Fixed threshold T (input units): object = q > q(T). */
int32_t oracle_q_thr_otsu(int32_t t_star, const or_params* p) {
    int64_t c = ((int64_t)(t_star + 1) * p->K + 255) / 256;
    return (int32_t)((int64_t)p->qmin + c);
}

int32_t oracle_q_thr_fixed(double T, const or_params* p) {
    float tf = (float)T;
    float rq = rintf(tf * p->r);
    double lo = (double)p->qmin - 1.0, hi = (double)p->qmax;
    double qd = (double)rq;
    int64_t qT;
    if (qd < lo)
        qT = (int64_t)p->qmin - 1;
    else if (qd > hi)
        qT = p->qmax;
    else
        qT = (int64_t)qd;
    return (int32_t)(qT + 1);
}

/* --------------------------------------------------------------- labelling */

typedef struct {
    uint64_t* a;
    uint64_t cap, head, tail; /* ring buffer */
} queue64;

static int q_push(queue64* q, uint64_t v) {
    if (q->tail - q->head == q->cap) {
        uint64_t ncap = q->cap ? q->cap * 2 : 1024;
        uint64_t* na = (uint64_t*)malloc(sizeof(uint64_t) * ncap);
        if (!na) return -1;
        for (uint64_t i = q->head; i < q->tail; ++i) na[i - q->head] = q->a[i % q->cap];
        free(q->a);
        q->a = na;
        q->tail -= q->head;
        q->head = 0;
        q->cap = ncap;
    }
    q->a[q->tail % q->cap] = v;
    q->tail++;
    return 0;
}

typedef struct {
    or_comp* a;
    uint64_t n, cap;
} compvec;

static or_comp* comp_new(compvec* c) {
    if (c->n == c->cap) {
        uint64_t ncap = c->cap ? c->cap * 2 : 64;
        or_comp* na = (or_comp*)realloc(c->a, sizeof(or_comp) * ncap);
        if (!na) return NULL;
        c->a = na;
        c->cap = ncap;
    }
    return &c->a[c->n++];
}

static inline int bit_at(const uint64_t* bits, uint64_t v) { return (int)((bits[v >> 6] >> (v & 63)) & 1u); }

/* Flood fill in raster order: the first voxel reached of each component is
 * its smallest linear index, which becomes the label.  comp[v] = component
 * number + 1 (0 = background).  Returns 0 or -1 (allocation). */
static int flood_fill(const uint64_t* bits, int64_t nx, int64_t ny, int64_t nz, int conn, uint32_t* comp,
                      compvec* comps) {
    int off[26][3], noff = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int manhattan = abs(dx) + abs(dy) + abs(dz);
                if (manhattan == 0) continue;
                if (conn == 6 && manhattan != 1) continue;
                off[noff][0] = dx;
                off[noff][1] = dy;
                off[noff][2] = dz;
                ++noff;
            }
    uint64_t N = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    queue64 q = {0};
    for (uint64_t v = 0; v < N; ++v) {
        if (!bit_at(bits, v) || comp[v]) continue;
        or_comp* c = comp_new(comps);
        if (!c) { free(q.a); return -1; }
        uint32_t id = (uint32_t)comps->n;
        memset(c, 0, sizeof *c);
        c->label = v;
        c->x0 = c->y0 = c->z0 = UINT32_MAX;
        comp[v] = id;
        if (q_push(&q, v)) { free(q.a); return -1; }
        while (q.head < q.tail) {
            uint64_t u = q.a[q.head % q.cap];
            q.head++;
            int64_t x = (int64_t)(u % (uint64_t)nx);
            int64_t y = (int64_t)((u / (uint64_t)nx) % (uint64_t)ny);
            int64_t z = (int64_t)(u / ((uint64_t)nx * (uint64_t)ny));
            or_comp* cc = &comps->a[id - 1];
            cc->size++;
            if ((uint32_t)x < cc->x0) cc->x0 = (uint32_t)x;
            if ((uint32_t)x + 1 > cc->x1) cc->x1 = (uint32_t)x + 1;
            if ((uint32_t)y < cc->y0) cc->y0 = (uint32_t)y;
            if ((uint32_t)y + 1 > cc->y1) cc->y1 = (uint32_t)y + 1;
            if ((uint32_t)z < cc->z0) cc->z0 = (uint32_t)z;
            if ((uint32_t)z + 1 > cc->z1) cc->z1 = (uint32_t)z + 1;
            for (int k = 0; k < noff; ++k) {
                int64_t xx = x + off[k][0], yy = y + off[k][1], zz = z + off[k][2];
                if (xx < 0 || yy < 0 || zz < 0 || xx >= nx || yy >= ny || zz >= nz) continue;
                uint64_t w = ((uint64_t)zz * (uint64_t)ny + (uint64_t)yy) * (uint64_t)nx + (uint64_t)xx;
                if (bit_at(bits, w) && !comp[w]) {
                    comp[w] = id;
                    if (q_push(&q, w)) { free(q.a); return -1; }
                }
            }
        }
        q.head = q.tail = 0;
    }
    free(q.a);
    return 0;
}

/* Keep rule (Sec. 4.2.1 keeps the largest object): LARGEST = most voxels,
 * ties to the smallest label (components are in label order); MIN_SIZE =
 * every component with size >= min_size. */
static void keep_components(or_comp* c, uint64_t n, int keep_mode, int64_t min_size) {
    if (keep_mode == OR_KEEP_LARGEST) {
        uint64_t best = 0, arg = UINT64_MAX;
        for (uint64_t i = 0; i < n; ++i)
            if (c[i].size > best) { best = c[i].size; arg = i; }
        for (uint64_t i = 0; i < n; ++i) c[i].kept = (i == arg);
    } else {
        for (uint64_t i = 0; i < n; ++i) c[i].kept = c[i].size >= (uint64_t)min_size;
    }
}

static uint64_t* mask_to_bits(const uint8_t* mask, uint64_t N) {
    uint64_t* bits = (uint64_t*)calloc((size_t)((N + 63) / 64), sizeof(uint64_t));
    if (!bits) return NULL;
    for (uint64_t v = 0; v < N; ++v)
        if (mask[v]) bits[v >> 6] |= 1ull << (v & 63);
    return bits;
}

/* Label a u8 mask (nonzero = object).  labels (nullable): int64 per voxel,
 * -1 for background.  comps: first comps_cap entries in label order.
 * Returns OR_OK, OR_ETRUNC (more components than comps_cap; *n_comps is the
 * true count) or OR_ENOMEM. */
int oracle_label(const uint8_t* mask, int64_t nx, int64_t ny, int64_t nz, int conn, int keep_mode,
                 int64_t min_size, int64_t* labels, uint8_t* keep, or_comp* comps, int64_t comps_cap,
                 uint64_t* n_comps) {
    uint64_t N = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    uint64_t* bits = mask_to_bits(mask, N);
    uint32_t* comp = (uint32_t*)calloc((size_t)N, sizeof(uint32_t));
    compvec cv = {0};
    if (!bits || !comp || flood_fill(bits, nx, ny, nz, conn, comp, &cv)) {
        free(bits); free(comp); free(cv.a);
        return OR_ENOMEM;
    }
    keep_components(cv.a, cv.n, keep_mode, min_size);
    for (uint64_t v = 0; v < N; ++v) {
        if (labels) labels[v] = comp[v] ? (int64_t)cv.a[comp[v] - 1].label : -1;
        if (keep) keep[v] = comp[v] ? (uint8_t)cv.a[comp[v] - 1].kept : 0;
    }
    *n_comps = cv.n;
    uint64_t m = cv.n < (uint64_t)comps_cap ? cv.n : (uint64_t)comps_cap;
    if (comps && m) memcpy(comps, cv.a, sizeof(or_comp) * m);
    free(bits); free(comp); free(cv.a);
    return cv.n > (uint64_t)comps_cap ? OR_ETRUNC : OR_OK;
}

/* ------------------------------------------------------------ rows/stream */

static void put_code(uint8_t* stream, uint64_t stream_cap, uint64_t idx, uint32_t u, int bytes) {
    uint64_t at = idx * (uint64_t)bytes;
    if (at + (uint64_t)bytes > stream_cap) return;
    for (int k = 0; k < bytes; ++k) stream[at + k] = (uint8_t)(u >> (8 * k));
}

/* Geometry section (Eq. 3): for every row that holds a kept voxel, the
 * leftmost kept x and one past the rightmost.  keep: u8 per voxel.
 * Returns the number of rows (rows written up to rows_cap). */
uint64_t oracle_rows(const uint8_t* keep, int64_t nx, int64_t ny, int64_t nz, or_row* rows, int64_t rows_cap) {
    uint64_t nr = 0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y) {
            const uint8_t* k = keep + (uint64_t)(z * ny + y) * (uint64_t)nx;
            int64_t xs = -1, xe = -1;
            for (int64_t x = 0; x < nx; ++x)
                if (k[x]) {
                    if (xs < 0) xs = x;
                    xe = x + 1;
                }
            if (xs < 0) continue;
            if (nr < (uint64_t)rows_cap) {
                rows[nr].z = (uint32_t)z;
                rows[nr].y = (uint32_t)y;
                rows[nr].xs = (uint32_t)xs;
                rows[nr].xe = (uint32_t)xe;
                rows[nr].code_off = 0;
                rows[nr].outlier_off = 0;
            }
            ++nr;
        }
    return nr;
}

/* Pixel section (Eq. 4): every voxel of every span, in row order, as
 * u = q - qmin in b bits little-endian, or the escape code followed (in the
 * outlier array) by the raw value.  Fills code_off/outlier_off of the rows.
 * Returns OR_OK or OR_ETRUNC (counts are still the full ones). */
int oracle_stream(const void* in, int dtype, int64_t nx, int64_t ny, const or_params* p, or_row* rows,
                  uint64_t n_rows, uint8_t* stream, uint64_t stream_cap_bytes, float* outliers,
                  uint64_t outliers_cap, uint64_t* n_codes, uint64_t* n_outliers) {
    int bytes = p->width_bits / 8;
    uint64_t nc = 0, no = 0;
    for (uint64_t i = 0; i < n_rows; ++i) {
        or_row* r = &rows[i];
        r->code_off = nc;
        r->outlier_off = no;
        uint64_t base = ((uint64_t)r->z * (uint64_t)ny + r->y) * (uint64_t)nx;
        for (uint32_t x = r->xs; x < r->xe; ++x) {
            float xv = voxel(in, dtype, base + x);
            int32_t q = code_of(xv, p);
            uint32_t u;
            if (is_outlier(xv, q, p)) {
                u = p->esc;
                if (no < outliers_cap) outliers[no] = xv;
                ++no;
            } else {
                u = (uint32_t)((int64_t)q - (int64_t)p->qmin);
            }
            put_code(stream, stream_cap_bytes, nc, u, bytes);
            ++nc;
        }
    }
    *n_codes = nc;
    *n_outliers = no;
    if (nc * (uint64_t)bytes > stream_cap_bytes || no > outliers_cap) return OR_ETRUNC;
    return OR_OK;
}

/* The normalised pixel section (Sec. 4.1.2, Eq. 1, feeding Sec. 4.2.3): the
 * 8-bit level of every voxel of every span, in the stream's order (rows in
 * table order, x from xs to xe - 1).  Eq. 1 scales intensities to 0..255; with
 * the minimum subtracted (reading R4) a voxel's level is the histogram bin of
 * its code, bin(q) = floor(256 (q - qmin) / K), computed exactly in integers,
 * so the section holds the levels the threshold was taken on.  The code is
 * the voxel's own q(x), escaped or not.  out receives n_codes bytes
 * (rows[i].code_off + x - xs).  Returns the quantiser status, or OR_EINVAL
 * for a row outside the volume. */
int oracle_section(const void* in, int dtype, int64_t nx, int64_t ny, int64_t nz, const or_params* p,
                   const or_row* rows, uint64_t n_rows, uint8_t* out) {
    if (p->status != OR_OK) return p->status;
    for (uint64_t i = 0; i < n_rows; ++i) {
        const or_row* r = &rows[i];
        if (r->z >= (uint64_t)nz || r->y >= (uint64_t)ny || r->xe > (uint64_t)nx || r->xs >= r->xe) return OR_EINVAL;
        const uint64_t base = ((uint64_t)r->z * (uint64_t)ny + r->y) * (uint64_t)nx;
        for (uint32_t x = r->xs; x < r->xe; ++x) {
            const float v = voxel(in, dtype, base + x);
            out[r->code_off + (x - r->xs)] = (uint8_t)bin_of(code_of(v, p), p);
        }
    }
    return OR_OK;
}

/* Background subtraction (Sec. 4.1.1): out = I - B voxel by voxel (op 0),
 * or out = I + B (op 1, the reverse process putting a decoded object back on
 * its background).  B holds bg_planes planes of ny * nx float32 values: one
 * plane for every z (bg_planes == 1) or one per z.  uint16 input (dtype 1)
 * is converted to float32 first (exactly).  One binary32 operation per
 * voxel.  Returns OR_EINVAL for a bad dtype, op or plane count. */
int oracle_background(const void* in, int dtype, const float* bg, int64_t bg_planes, int64_t nx, int64_t ny,
                      int64_t nz, int op, float* out) {
    if ((dtype != 0 && dtype != 1) || (op != 0 && op != 1) || (bg_planes != 1 && bg_planes != nz))
        return OR_EINVAL;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t v = (z * ny + y) * nx + x;
                int64_t b = ((bg_planes == 1 ? 0 : z) * ny + y) * nx + x;
                float i = dtype == 0 ? ((const float*)in)[v] : (float)((const uint16_t*)in)[v];
                out[v] = op == 0 ? i - bg[b] : i + bg[b];
            }
    return OR_OK;
}

/* Reverse process (Sec. 4.3): rebuild every row from the geometry section;
 * voxels outside the spans take `background`.  Returns OR_OK or OR_EINVAL on
 * an inconsistent stream. */
int oracle_decode(const or_row* rows, uint64_t n_rows, const uint8_t* stream, const float* outliers,
                  uint64_t n_outliers, const or_params* p, int64_t nx, int64_t ny, int64_t nz, float background,
                  float* out) {
    uint64_t N = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    for (uint64_t v = 0; v < N; ++v) out[v] = background;
    int bytes = p->width_bits / 8;
    uint64_t oi = 0;
    for (uint64_t i = 0; i < n_rows; ++i) {
        const or_row* r = &rows[i];
        if (r->z >= (uint64_t)nz || r->y >= (uint64_t)ny || r->xe > (uint64_t)nx || r->xs >= r->xe) return OR_EINVAL;
        uint64_t base = ((uint64_t)r->z * (uint64_t)ny + r->y) * (uint64_t)nx;
        if (r->outlier_off != oi) return OR_EINVAL;
        for (uint32_t x = r->xs; x < r->xe; ++x) {
            uint64_t idx = r->code_off + (x - r->xs);
            uint32_t u = 0;
            for (int k = 0; k < bytes; ++k) u |= (uint32_t)stream[idx * bytes + k] << (8 * k);
            float xh;
            if (u == p->esc) {
                if (oi >= n_outliers) return OR_EINVAL;
                xh = outliers[oi++];
            } else {
                int32_t q = (int32_t)((int64_t)u + (int64_t)p->qmin);
                xh = (float)q * p->w;
            }
            out[base + x] = xh;
        }
    }
    return oi == n_outliers ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------ fused */

/* The whole path on one volume, in the paper's order of dependence:
 * range -> error bound -> codes -> histogram -> threshold -> mask ->
 * components -> keep -> rows -> stream.  Buffers are caller-owned; a
 * buffer too small gives OR_ETRUNC with the full counts reported.
 * thr_mode OR_THR_SLICE thresholds each z-slice on its own, as the paper
 * thresholds each 2-D image (Sec. 4.1.3): two-class Otsu on the slice's
 * histogram over the volume's 256 bins, object = bins above the slice's
 * split; slice_thr (nz entries, may be NULL) receives the splits. */
int oracle_fused(const void* in, int dtype, int64_t nx, int64_t ny, int64_t nz, int eb_mode, double eb_value,
                 int thr_mode, double fixed_value, int conn, int keep_mode, int64_t min_size,
                 or_comp* comps, int64_t comps_cap, or_row* rows, int64_t rows_cap, uint8_t* stream,
                 int64_t stream_cap_bytes, float* outliers, int64_t outliers_cap, or_fused_info* info,
                 int32_t* slice_thr) {
    memset(info, 0, sizeof *info);
    info->otsu_bin = -1;
    double t0 = now_s(), t1;
    if (!in || nx <= 0 || ny <= 0 || nz <= 0 || (dtype != OR_F32 && dtype != OR_U16) ||
        (conn != 6 && conn != 26) || min_size < 1 || thr_mode < OR_THR_OTSU || thr_mode > OR_THR_SLICE)
        return info->q.status = info->seg_status = info->ext_status = OR_EINVAL;
    uint64_t N = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    float xmin, xmax;
    int st = oracle_range(in, dtype, N, &xmin, &xmax);
    if (st == OR_OK) st = oracle_resolve(xmin, xmax, eb_mode, eb_value, &info->q);
    else { info->q.status = st; info->q.xmin = info->q.xmax = 0.0f; }
    t1 = now_s(); info->stage_seconds[0] = t1 - t0; t0 = t1;
    if (st != OR_OK) return info->seg_status = info->ext_status = st;
    const or_params* p = &info->q;

    for (uint64_t v = 0; v < N; ++v) info->hist[bin_of(code_of(voxel(in, dtype, v), p), p)]++;
    t1 = now_s(); info->stage_seconds[1] = t1 - t0; t0 = t1;

    info->thresholds[0] = info->thresholds[1] = info->thresholds[2] = -1;
    if (thr_mode == OR_THR_OTSU) {
        info->flags |= oracle_otsu(info->hist, &info->otsu_bin);
        info->q_thr = oracle_q_thr_otsu(info->otsu_bin, p);
        info->thresholds[0] = info->otsu_bin;
        info->n_classes = 2;
    } else if (thr_mode == OR_THR_MULTI3 || thr_mode == OR_THR_MULTI4) {
        /* object = every class above the lowest threshold */
        info->n_classes = thr_mode == OR_THR_MULTI3 ? 3 : 4;
        info->flags |= oracle_multi_otsu(info->hist, info->n_classes, info->thresholds);
        info->otsu_bin = info->thresholds[0];
        info->q_thr = oracle_q_thr_otsu(info->otsu_bin, p);
    } else if (thr_mode == OR_THR_SLICE) {
        info->flags |= OR_FLAG_SLICE;
        info->n_classes = 2;
    } else {
        info->flags |= OR_FLAG_FIXED;
        info->q_thr = oracle_q_thr_fixed(fixed_value, p);
    }
    int32_t* sthr = NULL;
    if (thr_mode == OR_THR_SLICE) {
        sthr = (int32_t*)malloc((size_t)nz * sizeof(int32_t));
        if (!sthr) return info->seg_status = info->ext_status = OR_ENOMEM;
        const uint64_t plane = (uint64_t)nx * (uint64_t)ny;
        for (int64_t z = 0; z < nz; ++z) {
            uint64_t h[256] = {0};
            for (uint64_t v = (uint64_t)z * plane; v < (uint64_t)(z + 1) * plane; ++v)
                h[bin_of(code_of(voxel(in, dtype, v), p), p)]++;
            info->flags |= oracle_otsu(h, &sthr[z]);
            if (slice_thr) slice_thr[z] = sthr[z];
        }
    }
    uint64_t* bits = (uint64_t*)calloc((size_t)((N + 63) / 64), sizeof(uint64_t));
    if (!bits) {
        free(sthr);
        return info->seg_status = info->ext_status = OR_ENOMEM;
    }
    const uint64_t plane_n = (uint64_t)nx * (uint64_t)ny;
    for (uint64_t v = 0; v < N; ++v) {
        const int32_t q = code_of(voxel(in, dtype, v), p);
        const int object = sthr ? (int32_t)bin_of(q, p) > sthr[v / plane_n] : q >= info->q_thr;
        if (object) {
            bits[v >> 6] |= 1ull << (v & 63);
            info->n_mask++;
        }
    }
    free(sthr);
    t1 = now_s(); info->stage_seconds[2] = t1 - t0; t0 = t1;

    uint32_t* comp = (uint32_t*)calloc((size_t)N, sizeof(uint32_t));
    compvec cv = {0};
    if (!comp || flood_fill(bits, nx, ny, nz, conn, comp, &cv)) {
        free(bits); free(comp); free(cv.a);
        return info->seg_status = info->ext_status = OR_ENOMEM;
    }
    free(bits);
    t1 = now_s(); info->stage_seconds[3] = t1 - t0; t0 = t1;

    info->n_components = cv.n;
    if (cv.n > (uint64_t)comps_cap) {
        /* the keep rule needs the whole component table: stop after labelling,
         * reporting the number of components the table must hold */
        free(comp); free(cv.a);
        return info->seg_status = info->ext_status = OR_ETRUNC;
    }
    keep_components(cv.a, cv.n, keep_mode, min_size);
    uint32_t bb[6] = {UINT32_MAX, 0, UINT32_MAX, 0, UINT32_MAX, 0};
    for (uint64_t i = 0; i < cv.n; ++i) {
        if (!cv.a[i].kept) continue;
        info->n_kept++;
        info->n_kept_voxels += cv.a[i].size;
        if (cv.a[i].x0 < bb[0]) bb[0] = cv.a[i].x0;
        if (cv.a[i].x1 > bb[1]) bb[1] = cv.a[i].x1;
        if (cv.a[i].y0 < bb[2]) bb[2] = cv.a[i].y0;
        if (cv.a[i].y1 > bb[3]) bb[3] = cv.a[i].y1;
        if (cv.a[i].z0 < bb[4]) bb[4] = cv.a[i].z0;
        if (cv.a[i].z1 > bb[5]) bb[5] = cv.a[i].z1;
    }
    if (info->n_kept == 0) {
        info->flags |= OR_FLAG_EMPTY_ROI;
        memset(bb, 0, sizeof bb);
    }
    memcpy(info->bbox, bb, sizeof bb);
    if (comps && cv.n) memcpy(comps, cv.a, sizeof(or_comp) * cv.n);
    t1 = now_s(); info->stage_seconds[4] = t1 - t0; t0 = t1;

    /* rows from the kept components (all rows kept internally, so the
     * counts are complete even when the caller's buffers are too small) */
    or_row* all = (or_row*)malloc(sizeof(or_row) * (size_t)(nz * ny));
    if (!all) {
        free(comp); free(cv.a);
        return info->ext_status = OR_ENOMEM;
    }
    uint64_t nr = 0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y) {
            uint64_t base = (uint64_t)(z * ny + y) * (uint64_t)nx;
            int64_t xs = -1, xe = -1;
            for (int64_t x = 0; x < nx; ++x) {
                uint32_t c = comp[base + (uint64_t)x];
                if (c && cv.a[c - 1].kept) {
                    if (xs < 0) xs = x;
                    xe = x + 1;
                }
            }
            if (xs < 0) continue;
            all[nr].z = (uint32_t)z;
            all[nr].y = (uint32_t)y;
            all[nr].xs = (uint32_t)xs;
            all[nr].xe = (uint32_t)xe;
            ++nr;
        }
    free(comp);
    free(cv.a);
    info->n_rows = nr;
    t1 = now_s(); info->stage_seconds[5] = t1 - t0; t0 = t1;
    st = oracle_stream(in, dtype, nx, ny, p, all, nr, stream, (uint64_t)stream_cap_bytes, outliers,
                       (uint64_t)outliers_cap, &info->n_codes, &info->n_outliers);
    uint64_t m2 = nr < (uint64_t)rows_cap ? nr : (uint64_t)rows_cap;
    if (rows && m2) memcpy(rows, all, sizeof(or_row) * m2);
    free(all);
    if (nr > (uint64_t)rows_cap) st = OR_ETRUNC;
    info->stream_bytes = info->n_codes * (uint64_t)(p->width_bits / 8);
    t1 = now_s(); info->stage_seconds[6] = t1 - t0;
    for (int k = 0; k < 7; ++k) info->stage_seconds[7] += info->stage_seconds[k];
    info->ext_status = st;
    return st;
}

/* Absolute error-bounded quantisation of a pixel sequence (Sec. 4.2.3).
 * Input: D[0..m) 8-bit pixels (the normalised pixel section, Sec. 4.1.2) and
 * the tolerance E_abs.  The pixels are integers and so is the output, and
 * |Q - D| <= E for integers means |Q - D| <= floor(E): the tolerance used is
 * E = floor(E_abs).  With that E the floored midpoint keeps the bound, which
 * it does not for a fractional E >= 0.5 (e.g. D = {0, 3}, E = 1.5: the
 * tolerance intervals meet at 1.5 and the floor gives 1, 2 away from 3).
 *
 * The method cuts the sequence, from left to right, into the longest runs of
 * consecutive pixels that one value can represent within E, and gives every
 * pixel of a run that value.  One value fits a run exactly when the pixels'
 * tolerance intervals [D - E, D + E] share a point, i.e. when the run's
 * largest and smallest pixel differ by at most 2E; the shared points are
 * then [max - E, min + E], and the value written is the floor of that
 * interval's midpoint, floor((min + max) / 2), clipped to the 8-bit range
 * (a no-op here, since min and max are 8-bit).  So a run grows while
 * max - min <= 2E and the pixel that would break this starts the next run.
 * Exact integer arithmetic.  *n_groups receives the number of runs.  Returns
 * OR_EINVAL for a negative or NaN tolerance. */
static void abs_quantize_write(uint8_t* Q, uint64_t a, uint64_t b, int lo, int hi) {
    int q = (lo + hi) / 2; /* both >= 0: integer division is the floor */
    q = q < 0 ? 0 : q > 255 ? 255 : q;
    for (uint64_t j = a; j < b; ++j) Q[j] = (uint8_t)q;
}

int oracle_abs_quantize(const uint8_t* D, uint64_t m, double e_abs, uint8_t* Q, uint64_t* n_groups) {
    if (!(e_abs >= 0.0)) return OR_EINVAL;
    const int64_t E = e_abs >= 1024.0 ? 1024 : (int64_t)floor(e_abs);
    uint64_t start = 0, runs = 0;
    int lo = 0, hi = 0;
    for (uint64_t i = 0; i < m; ++i) {
        const int d = D[i];
        if (i == start) {
            lo = hi = d;
            continue;
        }
        const int nlo = d < lo ? d : lo, nhi = d > hi ? d : hi;
        if ((int64_t)(nhi - nlo) > 2 * E) {
            abs_quantize_write(Q, start, i, lo, hi);
            ++runs;
            start = i;
            lo = hi = d;
        } else {
            lo = nlo;
            hi = nhi;
        }
    }
    if (m > 0) {
        abs_quantize_write(Q, start, m, lo, hi);
        ++runs;
    }
    *n_groups = runs;
    return OR_OK;
}

/* ---- Huffman coding of a byte sequence ----
 * Code lengths by Huffman's construction (1952) over the byte counts, with a
 * fixed order for equal weights: the leaves sorted by (count, byte value)
 * and the merged nodes, created in order of non-decreasing weight, form two
 * queues; each step takes the two lightest heads, a leaf before a merged
 * node of the same weight.  A single used byte gets length 1.  Lengths above
 * 32 bits are refused (OR_ERANGE).  Canonical codes: within a length, codes
 * increase with the byte value, and the first code of length L follows the
 * last of length L - 1 shifted left (the assignment of RFC 1951, 3.2.2).
 * Format: the input is cut into blocks of 4096 bytes; block b is written
 * from 32-bit word block_off[b] of the payload, its codes one after another
 * from the most significant bit of each word down, zero bits up to the next
 * word; block_off[nblocks] is the payload length in words.
 * Sub-block index (optional): each block is also cut into 16 sub-blocks of
 * 256 input bytes, and sub_bits[16 b + k] is the number of code bits of
 * sub-block k of block b (0 for sub-blocks past the input's end).  The codes
 * of consecutive sub-blocks follow each other with no padding, so the payload
 * is the same with or without the index; sub-block k starts at bit
 * sub_bits[16 b] + ... + sub_bits[16 b + k - 1] of its block, which lets a
 * decoder start at every sub-block at once. */
#define OR_HUFF_BLOCK 4096
#define OR_HUFF_SUB 256
#define OR_HUFF_SUBS (OR_HUFF_BLOCK / OR_HUFF_SUB)

int oracle_huff_lengths(const uint64_t hist[256], uint8_t len[256]) {
    int sym[256], ns = 0;
    for (int i = 0; i < 256; ++i) {
        len[i] = 0;
        if (hist[i]) sym[ns++] = i;
    }
    if (ns == 0) return OR_OK;
    if (ns == 1) {
        len[sym[0]] = 1;
        return OR_OK;
    }
    for (int i = 1; i < ns; ++i) /* insertion sort by (count, byte) */
        for (int j = i; j > 0 && hist[sym[j]] < hist[sym[j - 1]]; --j) {
            int t = sym[j];
            sym[j] = sym[j - 1];
            sym[j - 1] = t;
        }
    /* nodes 0..ns-1: the leaves in queue order; ns..2ns-2: merged nodes */
    uint64_t w[511];
    int parent[511];
    for (int i = 0; i < ns; ++i) w[i] = hist[sym[i]];
    int lq = 0, mq = ns, next = ns;
    while (next < 2 * ns - 1) {
        int pick[2];
        for (int k = 0; k < 2; ++k) {
            if (lq < ns && (mq >= next || w[lq] <= w[mq])) pick[k] = lq++;
            else pick[k] = mq++;
        }
        w[next] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = parent[pick[1]] = next;
        ++next;
    }
    int depth[511];
    depth[2 * ns - 2] = 0;
    for (int i = 2 * ns - 3; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
    for (int i = 0; i < ns; ++i) {
        if (depth[i] > 32) return OR_ERANGE;
        len[sym[i]] = (uint8_t)depth[i];
    }
    return OR_OK;
}

static void huff_codes(const uint8_t len[256], uint32_t code[256]) {
    uint32_t bl_count[34] = {0}, next_code[34] = {0};
    for (int i = 0; i < 256; ++i) bl_count[len[i]]++;
    bl_count[0] = 0;
    uint64_t c = 0;
    for (int bits = 1; bits <= 32; ++bits) {
        c = (c + bl_count[bits - 1]) << 1;
        next_code[bits] = (uint32_t)c;
    }
    for (int i = 0; i < 256; ++i) code[i] = len[i] ? next_code[len[i]]++ : 0u;
}

/* Encode: lengths from the counts of `in`, then the blocks.  block_off has
 * nblocks + 1 entries; sub_bits (16 nblocks entries) may be NULL.  OR_ETRUNC
 * (and *total_words) when the payload does not fit cap_words. */
int oracle_huff_encode(const uint8_t* in, uint64_t n, uint8_t len[256], uint64_t* block_off, uint32_t* payload,
                       uint64_t cap_words, uint64_t* total_words, uint16_t* sub_bits) {
    uint64_t hist[256] = {0};
    for (uint64_t i = 0; i < n; ++i) hist[in[i]]++;
    int st = oracle_huff_lengths(hist, len);
    if (st != OR_OK) return st;
    uint32_t code[256];
    huff_codes(len, code);
    const uint64_t nb = (n + OR_HUFF_BLOCK - 1) / OR_HUFF_BLOCK;
    uint64_t word = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        block_off[b] = word;
        uint64_t bits = 0;
        const uint64_t e = (b + 1) * OR_HUFF_BLOCK < n ? (b + 1) * OR_HUFF_BLOCK : n;
        for (uint64_t i = b * OR_HUFF_BLOCK; i < e; ++i) bits += len[in[i]];
        if (sub_bits) {
            for (int k = 0; k < OR_HUFF_SUBS; ++k) {
                uint64_t sb = 0;
                for (uint64_t i = b * OR_HUFF_BLOCK + (uint64_t)k * OR_HUFF_SUB;
                     i < e && i < b * OR_HUFF_BLOCK + (uint64_t)(k + 1) * OR_HUFF_SUB; ++i)
                    sb += len[in[i]];
                sub_bits[b * OR_HUFF_SUBS + k] = (uint16_t)sb; /* at most 256 * 32 = 8192 */
            }
        }
        const uint64_t words = (bits + 31) / 32;
        if (word + words <= cap_words) {
            for (uint64_t k = 0; k < words; ++k) payload[word + k] = 0u;
            uint64_t p = 0; /* bit position from the block's first bit, most significant first */
            for (uint64_t i = b * OR_HUFF_BLOCK; i < e; ++i) {
                const int L = len[in[i]];
                for (int k = L - 1; k >= 0; --k, ++p)
                    if ((code[in[i]] >> k) & 1u) payload[word + p / 32] |= 0x80000000u >> (p % 32);
            }
        }
        word += words;
    }
    block_off[nb] = word;
    *total_words = word;
    return word > cap_words ? OR_ETRUNC : OR_OK;
}

/* One code at bit p of a block's bits (nbits of them); the byte, and p
 * moved past it; -1 when the bits match no code before their end. */
static int huff_next(const uint8_t len[256], const uint32_t code[256], const uint32_t* words, uint64_t nbits,
                     uint64_t* p) {
    uint32_t c = 0;
    for (int L = 1; L <= 32; ++L) {
        if (*p >= nbits) return -1;
        c = (c << 1) | ((words[*p / 32] >> (31 - *p % 32)) & 1u);
        ++*p;
        for (int s = 0; s < 256; ++s)
            if (len[s] == L && code[s] == c) return s;
    }
    return -1;
}

/* Decode n bytes; OR_EINVAL on lengths that are no prefix code, offsets that
 * decrease or pass the payload, or bits that match no code.  With sub_bits,
 * every sub-block is decoded from its own start, and a sub-block whose codes
 * do not take exactly its stated bits (or stated bits past the block's
 * words) is OR_EINVAL too. */
int oracle_huff_decode(const uint8_t len[256], const uint64_t* block_off, const uint32_t* payload,
                       uint64_t payload_words, uint64_t n, uint8_t* out, const uint16_t* sub_bits) {
    uint32_t code[256];
    double kraft = 0.0;
    int used = 0;
    for (int i = 0; i < 256; ++i)
        if (len[i]) {
            if (len[i] > 32) return OR_EINVAL;
            kraft += ldexp(1.0, -len[i]);
            ++used;
        }
    if (n > 0 && used == 0) return OR_EINVAL;
    if (kraft > 1.0) return OR_EINVAL;
    huff_codes(len, code);
    const uint64_t nb = (n + OR_HUFF_BLOCK - 1) / OR_HUFF_BLOCK;
    if (nb > 0 && block_off[0] != 0) return OR_EINVAL;
    for (uint64_t b = 0; b < nb; ++b) {
        if (block_off[b + 1] < block_off[b] || block_off[b + 1] > payload_words) return OR_EINVAL;
        const uint32_t* words = payload + block_off[b];
        const uint64_t nbits = (block_off[b + 1] - block_off[b]) * 32;
        const uint64_t i0 = b * OR_HUFF_BLOCK, e = i0 + OR_HUFF_BLOCK < n ? i0 + OR_HUFF_BLOCK : n;
        if (!sub_bits) {
            uint64_t p = 0;
            for (uint64_t i = i0; i < e; ++i) {
                const int s = huff_next(len, code, words, nbits, &p);
                if (s < 0) return OR_EINVAL;
                out[i] = (uint8_t)s;
            }
            continue;
        }
        uint64_t start = 0; /* the sub-block's first bit */
        for (int k = 0; k < OR_HUFF_SUBS; ++k) {
            const uint64_t s0 = i0 + (uint64_t)k * OR_HUFF_SUB;
            const uint64_t s1 = s0 + OR_HUFF_SUB < e ? s0 + OR_HUFF_SUB : e;
            const uint64_t stated = sub_bits[b * OR_HUFF_SUBS + k];
            if (start + stated > nbits) return OR_EINVAL;
            uint64_t p = start;
            for (uint64_t i = s0; i < s1; ++i) {
                const int s = huff_next(len, code, words, start + stated, &p);
                if (s < 0) return OR_EINVAL;
                out[i] = (uint8_t)s;
            }
            if (p != start + stated) return OR_EINVAL;
            start += stated;
        }
    }
    return OR_OK;
}

/* struct sizes, so the Python side can check its mirrors */
void oracle_sizes(int64_t* out) {
    out[0] = (int64_t)sizeof(or_params);
    out[1] = (int64_t)sizeof(or_comp);
    out[2] = (int64_t)sizeof(or_row);
    out[3] = (int64_t)sizeof(or_fused_info);
}
