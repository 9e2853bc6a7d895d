/*
 * roix.h - C ABI of the MI355X ROI reduction library (libroix.so).
 *
 * The library runs the data-parallel reduction stage of ROIX-Comp
 * (arXiv 2602.15917) on one gfx950 GPU, for a 3-D volume of float32 or
 * uint16 voxels:
 *
 *   quantise  error-bounded codes, |x - xhat| <= E_abs for every voxel
 *             (Sec. 4.2.3, problem statement of the absolute error-bounded
 *             quantiser: input pixels and a positive tolerance E_abs)
 *   segment   8-bit normalisation to a 256-bin histogram (Sec. 4.1.2, Eq. 1),
 *             Otsu threshold (Sec. 4.1.3), binary mask (Sec. 4.1.4, Eq. 2),
 *             3-D connected components and the largest object / a minimum
 *             size (Sec. 4.2.1, volumetric form of the contour step)
 *   extract   per row the leftmost and rightmost retained voxel,
 *             G(i) = [i, x_start, x_end] (Sec. 4.2.2, Eq. 3), and the codes of
 *             the voxels in between, P(i) (Sec. 4.2.2, Eq. 4), as one packed
 *             stream with an index table (the 1-D array of Sec. 4.3)
 *
 * Conventions shared by every call:
 *  - Volumes are C-contiguous [nz][ny][nx]; linear index v = (z*ny + y)*nx + x.
 *  - d_* arguments are device pointers (hipMalloc'ed memory of the current
 *    device, e.g. torch tensors); every input and output buffer is owned by
 *    the caller.  The context owns only its scratch arena, allocated once in
 *    roix_ctx_create.  No call allocates device memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *    are asynchronous: they validate their arguments, enqueue kernels and
 *    return.  Results, including the status fields of the info structs, are
 *    valid after the stream is synchronised.
 *  - Argument errors are returned synchronously and enqueue nothing.  Data
 *    errors are written to the `status` field of the device info structs:
 *      ROIX_EINVAL  a NaN/Inf voxel; an error bound that is not a positive
 *                   normal float32 after resolution (e.g. a relative bound
 *                   on a constant volume); a code outside [qmin, qmax]
 *                   given to roix_segment
 *      ROIX_ERANGE  |x / (2 eb)| exceeds 2^24 (codes would not be exact)
 *      ROIX_ENOMEM  more foreground runs than the scratch arena can hold
 *      ROIX_ETRUNC  an output buffer is too small; the counts still report
 *                   the required sizes (the component table is needed by
 *                   the keep rule, so a short component table stops the
 *                   path after labelling)
 *    On a data error the contents of output buffers are unspecified, except
 *    the info structs.
 *  - A context is not thread-safe: use one context per host thread (or
 *    serialise), and do not run two calls on one context concurrently on
 *    different streams.
 *  - No C++ exception crosses this interface.
 */
#ifndef ROIX_H
#define ROIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROIX_OK = 0,
    ROIX_EINVAL = 1,
    ROIX_ERANGE = 2,
    ROIX_ENOMEM = 3,
    ROIX_ETRUNC = 4,
    ROIX_EDEVICE = 5,
    ROIX_EBUSY = 6,
    ROIX_ESEQ = 7
} roix_status;

typedef enum { ROIX_F32 = 0, ROIX_U16 = 1 } roix_dtype;

typedef struct {
    int64_t nx, ny, nz; /* each >= 1; nx*ny*nz <= 2^33 */
} roix_dims;

/* Error bound (Sec. 4.2.3: a positive absolute tolerance).  REL means
 * value * (xmax - xmin) of the volume.  The bound actually enforced, eb32,
 * is the largest float32 not above the requested one. */
typedef enum { ROIX_EB_ABS = 0, ROIX_EB_REL = 1 } roix_eb_mode;
typedef struct {
    int32_t mode; /* roix_eb_mode */
    int32_t pad;
    double value; /* > 0, finite */
} roix_eb;

/* ROI criterion.  OTSU: two-class Otsu (1979) on the 256-bin histogram of
 * the codes (Sec. 4.1.3); the object class is the bins strictly above the
 * split.  MULTI_OTSU: the multi-level Otsu of Liao, Chen & Chung (2001)
 * that Sec. 4.1.3 names, with `classes` = 3 or 4 classes (0 means 3): the
 * thresholds t1 < .. < t_{K-1} (bins 0..254, class k = bins t_k + 1 ..
 * t_{k+1}) maximise sum_k S_k^2 / W_k (W_k voxels and S_k the bin sum of
 * class k, the between-class variance up to a factor and a constant),
 * evaluated in binary64 in class order; tuples with an empty class are
 * skipped and the first maximum in lexicographic order wins; the object is
 * every class above the lowest threshold.  OTSU_SLICE: each z-slice is
 * thresholded on its own, as the paper thresholds each 2-D image: two-class
 * Otsu on the slice's histogram over the volume's 256 bins, object = bins
 * above the slice's split (roix_fused and roix_fused_batch only; the splits
 * go to roix_fused_out.d_slice_thr).  FIXED: voxels whose code is
 * above the code of `fixed_value` (input units) are object.  Connectivity 6
 * or 26.  LARGEST keeps the component with the most voxels (ties: smallest
 * label); MIN_SIZE keeps every component of at least `min_size` voxels. */
typedef enum { ROIX_THR_OTSU = 0, ROIX_THR_FIXED = 1, ROIX_THR_MULTI_OTSU = 2, ROIX_THR_OTSU_SLICE = 3 } roix_thr_mode;
typedef enum { ROIX_KEEP_MIN_SIZE = 0, ROIX_KEEP_LARGEST = 1 } roix_keep_mode;
typedef struct {
    int32_t thr;          /* roix_thr_mode */
    int32_t connectivity; /* 6 | 26 */
    double fixed_value;   /* FIXED only; finite */
    int32_t keep;         /* roix_keep_mode */
    int32_t classes;      /* MULTI_OTSU only: 3 or 4 (0 = 3); otherwise ignored */
    int64_t min_size;     /* MIN_SIZE only; >= 1 */
} roix_criterion;

/* Resolved quantiser: q(x) = rint(x * r) (float32 multiply, ties to even),
 * xhat = (float)q * w, outlier <=> !(|x - xhat| <= eb32); w = 2*eb32,
 * r = 1/w rounded once.  Codes are stored as u = q - qmin in width_bits
 * (8 if K <= 255, 16 if K <= 65535, else 32, K = qmax - qmin + 1); the
 * escape code esc = 2^width_bits - 1 marks an outlier.
 * n_outliers counts every voxel (roix_quantize); roix_fused does not
 * compute it and sets ROIX_NOT_COMPUTED. */
#define ROIX_NOT_COMPUTED UINT64_MAX
typedef struct {
    int32_t status;
    float xmin, xmax; /* value range; xmin <= xmax in IEEE total order */
    float eb32, w, r;
    int32_t qmin, qmax;
    int64_t K;
    int32_t width_bits;
    uint32_t esc;
    uint64_t n_outliers;
} roix_quant_info; /* 56 bytes */

#define ROIX_FLAG_DEGENERATE_HISTOGRAM 1u /* no Otsu split has two non-empty classes */
#define ROIX_FLAG_EMPTY_ROI 2u            /* no component kept */
#define ROIX_FLAG_FIXED_THRESHOLD 4u
#define ROIX_FLAG_PER_SLICE 8u            /* OTSU_SLICE: per-slice splits (otsu_bin -1, q_thr 0) */

/* hist[t] counts voxels with floor(256 (q - qmin) / K) == t.  otsu_bin = t*
 * (the lowest threshold for MULTI_OTSU; -1 for FIXED); the mask is
 * q >= q_thr.  thresholds: t* for OTSU (n_classes 2), t1 < t2 (< t3) for
 * MULTI_OTSU (n_classes 3 or 4), -1 in unused slots and for FIXED
 * (n_classes 0); with no valid split every threshold is 255.  bbox is the
 * half-open box [x0,x1) x [y0,y1) x [z0,z1) of the kept components (all 0
 * when none). */
typedef struct {
    int32_t status;
    int32_t otsu_bin;
    int32_t q_thr;
    uint32_t flags;
    uint64_t hist[256];
    uint64_t n_mask;        /* object voxels */
    uint64_t n_components;
    uint64_t n_kept;        /* kept components */
    uint64_t n_kept_voxels;
    uint32_t bbox[6];       /* x0, x1, y0, y1, z0, z1 */
    int32_t thresholds[3];
    int32_t n_classes;
} roix_seg_info;

/* One connected component, in ascending label order.  label = smallest
 * linear voxel index of the component. */
typedef struct {
    uint64_t label;
    uint64_t size;
    uint32_t x0, x1, y0, y1, z0, z1; /* half-open */
    uint32_t kept;
    uint32_t pad;
} roix_component; /* 48 bytes */

/* Geometry section entry (Eq. 3) of row (z, y): the span [xs, xe) covers
 * every voxel between the leftmost and the rightmost kept voxel, so
 * n_i = xe - xs.  Its codes are stream[code_off .. code_off + n_i) (in
 * codes, not bytes); its outliers start at outliers[outlier_off].  Rows
 * without a kept voxel are omitted; rows are in raster order (z, then y). */
typedef struct {
    uint32_t z, y, xs, xe;
    uint64_t code_off, outlier_off;
} roix_row; /* 32 bytes */

typedef struct {
    int32_t status;
    int32_t pad;
    uint64_t n_rows;
    uint64_t n_codes;
    uint64_t n_outliers;
    uint64_t stream_bytes; /* n_codes * width_bits / 8 */
} roix_extract_info;

/* Outputs of roix_extract / roix_fused.  Any info pointer may be NULL.
 * Caps are element counts (bytes for the stream). */
typedef struct {
    roix_row* d_rows;
    int64_t rows_cap;
    void* d_stream;
    int64_t stream_cap_bytes;
    float* d_outliers;
    int64_t outliers_cap;
    roix_component* d_comps;
    int64_t comps_cap;
    roix_quant_info* d_qinfo;
    roix_seg_info* d_sinfo;
    roix_extract_info* d_einfo;
    int32_t* d_slice_thr; /* nz: each slice's Otsu split (255: none) for OTSU_SLICE; may be NULL */
} roix_fused_out;

typedef struct roix_ctx roix_ctx;

/* Create a context on `device` with a scratch arena of `scratch_bytes`
 * (0 = 1 GiB).  The arena holds the per-voxel 8-bit bin proxy (N bytes),
 * the row bitmask (N/8 bytes), per-row tables and the run tables of the
 * labelling (17 bytes per foreground run); roix_scratch_bytes gives the size
 * that never yields ROIX_ENOMEM for a volume.  Errors: ROIX_EINVAL (bad
 * device / NULL out), ROIX_ENOMEM (allocation failed), ROIX_EDEVICE. */
roix_status roix_ctx_create(int device, size_t scratch_bytes, roix_ctx** out);
roix_status roix_ctx_destroy(roix_ctx* ctx);

/* Worst-case scratch for a volume (every row holding ceil(nx/2) runs).
 * Returns 0 for invalid dims. */
size_t roix_scratch_bytes(roix_dims dims, roix_dtype dtype, const roix_criterion* crit);

/* Worst-case output capacities: rows <= nz*ny, stream <= 4*N bytes,
 * outliers <= N, components <= N (6-connectivity) or
 * ceil(nx/2)*ceil(ny/2)*ceil(nz/2) (26-connectivity).  Any pointer may be
 * NULL.  A caller that allocates these never sees ROIX_ETRUNC.  The
 * component bound (and so the criterion argument) is there because the
 * fused call also writes the component table, whose worst case depends on
 * the connectivity. */
roix_status roix_bounds(roix_dims dims, roix_dtype dtype, const roix_criterion* crit, int64_t* max_rows,
                        int64_t* max_stream_bytes, int64_t* max_outliers, int64_t* max_components);

/* Quantise only (Sec. 4.2.3): d_codes[v] = q(x_v) (int32, N entries);
 * d_outlier_bits (nullable) bit v%32 of word v/32 set for outliers
 * (ceil(N/32) words); d_qinfo receives the resolved quantiser and the
 * outlier count.  Errors: ROIX_EINVAL (NULL ctx/d_in/d_codes/d_qinfo, bad
 * dims/dtype/eb). */
roix_status roix_quantize(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                          int32_t* d_codes, uint32_t* d_outlier_bits, roix_quant_info* d_qinfo, void* stream);

/* Segment codes (Sec. 4.1.2-4.2.1): histogram, threshold, mask, 3-D
 * components, keep rule.  d_codes and d_qinfo as written by roix_quantize.
 * d_keep (N bytes): 1 for voxels of kept components.  d_labels (nullable,
 * N int64): component label, -1 for background.  d_comps: components in
 * label order (comps_cap entries).  Errors: ROIX_EINVAL (NULL
 * ctx/d_codes/d_qinfo/crit/d_keep/d_sinfo, bad dims or criterion). */
roix_status roix_segment(roix_ctx* ctx, const int32_t* d_codes, roix_dims dims, const roix_quant_info* d_qinfo,
                         const roix_criterion* crit, uint8_t* d_keep, int64_t* d_labels, roix_component* d_comps,
                         int64_t comps_cap, roix_seg_info* d_sinfo, void* stream);

/* Extract (Sec. 4.2.2): rows of d_keep and the packed codes of the voxels of
 * d_in inside each span, recomputed with the quantiser in d_qinfo.  Uses
 * out->d_rows, d_stream, d_outliers and d_einfo (the component and
 * segmentation fields are ignored).  It takes the input rather than the code
 * array of roix_quantize: a code is a function of its voxel and the
 * resolved quantiser alone, so re-reading the span voxels (and recomputing
 * the outlier test) gives the same codes while reading only the spans,
 * where a code array would cost 4 bytes per voxel written and read again;
 * outputs equal roix_fused's either way.  Errors: ROIX_EINVAL (NULL
 * arguments, bad dims/dtype). */
roix_status roix_extract(roix_ctx* ctx, const void* d_in, roix_dtype dtype, const uint8_t* d_keep,
                         roix_dims dims, const roix_quant_info* d_qinfo, const roix_fused_out* out,
                         void* stream);

/* The whole path in one call: range, bound, codes, histogram, threshold,
 * components, keep, rows, stream.  No per-voxel code, mask or label array
 * is materialised.  Output equals roix_quantize + roix_segment +
 * roix_extract on the same input.  Errors: ROIX_EINVAL (NULL ctx/d_in/out,
 * bad dims/dtype/eb/criterion), ROIX_ENOMEM (scratch arena smaller than the
 * fixed per-voxel part), ROIX_EDEVICE (launch failure). */
roix_status roix_fused(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                       const roix_criterion* crit, const roix_fused_out* out, void* stream);

/* No-allocation form of roix_fused, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It needs no context: its scratch arena is a fixed array
 * of ROIX_NOALLOC_SCRATCH_BYTES compiled into the library, one copy per GPU,
 * held until the process ends.  It runs on the current device (the stream
 * must belong to it) with the launch parameters of a new context, and
 * enqueues exactly the kernels of roix_fused, so its outputs equal
 * roix_fused's bit for bit.
 *  - Limit: the volume's worst-case scratch (roix_scratch_bytes) must not
 *    exceed ROIX_NOALLOC_SCRATCH_BYTES (64 MiB: e.g. 128^3 float32 volumes);
 *    a larger volume returns ROIX_ENOMEM synchronously and enqueues nothing.
 *  - Every call on one GPU shares that GPU's array, and each call resets the
 *    state it reads at its start: calls that overlap on one GPU (two streams,
 *    two host threads) race.  Serialise them, e.g. on one stream.
 *  - Errors: as roix_fused (ROIX_EINVAL for bad arguments), ROIX_ENOMEM (too
 *    large, see above), ROIX_EDEVICE (the array's address could not be
 *    resolved on this device, or a launch failed).
 *  - Allocates nothing: no hipMalloc, hipFree or allocating library call. */
#define ROIX_NOALLOC_SCRATCH_BYTES (64ull << 20)
roix_status roix_fused_noalloc(const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                               const roix_criterion* crit, const roix_fused_out* out, void* stream);

/* Decode: the reverse process of Sec. 4.3, which rebuilds the volume from
 * the geometry section (Eq. 3, the row table), the pixel section (Eq. 4,
 * the code stream) and the outlier values, as written by roix_extract or
 * roix_fused.  Voxel (z, y, x) inside the span [xs, xe) of a row takes
 * (float)(u + qmin) * w for its code u (float32 multiply), or, for the
 * escape code, the next outlier value of its row in order of x (starting at
 * the row's outlier_off); every other voxel takes `background`.
 *   d_rows, rows_cap          the row table and its capacity (entries)
 *   d_stream, stream_cap_bytes the code stream and its capacity (bytes)
 *   d_outliers, outliers_cap  outlier values and their capacity
 *   d_qinfo                   the quantiser (qmin, w, width_bits, esc)
 *   d_einfo                   the counts n_rows, n_codes, n_outliers
 *   d_out                     N float32, C order [nz][ny][nx]; every voxel
 *                             is written
 *   d_dinfo                   device: status and the counts used
 * All device pointers, caller-owned; the call reads the counts on the
 * device, so it can follow roix_fused on the same stream without a host
 * synchronisation.  The context's arena holds a row descriptor of 32 bytes
 * per row (ny * nz) while the call runs.
 * d_dinfo->status is ROIX_EINVAL (and d_out unspecified) when the inputs are
 * not one consistent extraction: the quant or extract status is not OK, a
 * count exceeds its capacity, the width is not 8/16/32 or esc not 2^b - 1,
 * a row lies outside the volume or has xs >= xe or codes beyond n_codes,
 * rows are not in strictly increasing raster order, the first row's
 * outlier_off is not 0, or a row's outlier_off plus its escapes is not the
 * next row's (n_outliers for the last row).
 * Errors: ROIX_EINVAL (NULL ctx/d_qinfo/d_einfo/d_out/d_dinfo, bad dims,
 * negative or unbacked capacities, misaligned buffers), ROIX_ENOMEM (arena
 * smaller than the row descriptors), ROIX_EDEVICE. */
typedef struct {
    int32_t status;
    int32_t pad;
    uint64_t n_rows;
    uint64_t n_codes;
    uint64_t n_outliers;
} roix_decode_info; /* 32 bytes */
roix_status roix_decode(roix_ctx* ctx, const roix_row* d_rows, int64_t rows_cap, const void* d_stream,
                        int64_t stream_cap_bytes, const float* d_outliers, int64_t outliers_cap,
                        const roix_quant_info* d_qinfo, const roix_extract_info* d_einfo, roix_dims dims,
                        float background, float* d_out, roix_decode_info* d_dinfo, void* stream);

/* Background subtraction (Sec. 4.1.1): the output image is the input minus
 * a background reference, voxel by voxel, M = I - B; and its inverse for the
 * reverse process (Sec. 4.3), which puts the reconstructed object back on
 * the background, I' = M' + B.
 *   d_in       N voxels, C order [nz][ny][nx]: float32, or uint16 (SUBTRACT
 *              only; converted exactly to float32 first)
 *   d_bg       float32 reference, bg_planes planes of ny * nx voxels: 1 (the
 *              same calibration plane for every z) or nz (a reference volume)
 *   op         ROIX_BG_SUBTRACT: out = in - bg;  ROIX_BG_ADD: out = in + bg
 *   d_out      N float32; may be d_in itself when the input is float32 (in
 *              place), must not overlap it otherwise, nor the reference
 * One float32 operation per voxel, rounded to nearest even, so the output
 * is exact to the bit.  Subtracting before roix_fused (on the same stream)
 * runs the whole path on M; decoding and adding the reference back rebuilds
 * I within the error bound plus the roundings of the two operations.  All
 * pointers are device memory owned by the caller; asynchronous on `stream`.
 * Errors: ROIX_EINVAL (NULL arguments, bad dims or dtype, ADD on uint16,
 * bg_planes not 1 or nz, misaligned or overlapping buffers), ROIX_EDEVICE. */
typedef enum { ROIX_BG_SUBTRACT = 0, ROIX_BG_ADD = 1 } roix_bg_op;
roix_status roix_background(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, const float* d_bg,
                            int64_t bg_planes, roix_bg_op op, float* d_out, void* stream);

/* The fused path of roix_fused on M = I - B (background subtraction,
 * Sec. 4.1.1, then the whole path): the outputs are those of
 * roix_background followed by roix_fused on its output, bit for bit.  With
 * an absolute bound, rows of whole 64-voxel words and 16-byte aligned image
 * and reference, the subtraction is folded into the passes that read the
 * image (the range/code pass reads I and B; outlier values are gathered as
 * I - B), so M is not written.  M goes to d_work only where a stage must read
 * it: when the code range exceeds 2^15 codes (the 1-byte proxy flow) or when
 * the code emit meets chunks of many short spans.  Any other case
 * (a relative bound, other row lengths, OTSU_SLICE) subtracts into d_work
 * first and runs roix_fused on it.
 *   d_in      N float32 image
 *   d_bg      float32 reference of bg_planes planes (1 or nz), as
 *             roix_background
 *   d_work    N float32, caller-owned workspace overlapping neither d_in
 *             nor d_bg; its contents afterwards are unspecified
 * Other arguments, outputs, arena use and errors as roix_fused; also
 * ROIX_EINVAL for bg_planes not 1 or nz, a NULL reference or workspace, or
 * overlapping buffers. */
roix_status roix_fused_background(roix_ctx* ctx, const float* d_in, roix_dims dims, const float* d_bg,
                                  int64_t bg_planes, roix_eb eb, const roix_criterion* crit,
                                  const roix_fused_out* out, float* d_work, void* stream);

/* The normalised 8-bit pixel section of an extraction (Sec. 4.1.2, Eq. 1,
 * which maps each voxel onto 0..255 with the volume's own range): for span
 * voxel i of a completed roix_fused (or roix_extract) call, in the order of
 * its code stream, section[i] = floor(256 (q - qmin) / K), the voxel's
 * quantisation code q put on the 256 levels of the threshold histogram (so
 * a kept voxel's level is above otsu_bin and a masked-out voxel's is not).
 * This is the 8-bit sequence the paper's quantiser (roix_abs_quantize) takes.
 * The levels come from the stored codes (u = q - qmin); an escaped code's
 * voxel is read from d_in, found through the row table, and requantised.
 *   d_in       the volume the extraction was made from (dims, dtype as there)
 *   out        that call's outputs: d_qinfo, d_einfo, d_rows (rows_cap) and
 *              d_stream (stream_cap_bytes, 16-byte aligned) are read
 *   d_section  out: section_cap bytes, 16-byte aligned; n_codes are written
 *   d_info     device: status, n_codes
 * info.status: the extraction's own error if it had one (nothing written),
 * ROIX_ETRUNC when n_codes > section_cap (nothing written), ROIX_EINVAL when
 * the row table or the stream is not whole or does not cover every code.
 * The context's arena holds a list of the escaped codes while the call runs
 * (32 KB of counts, then 8 bytes per escape, split evenly over up to 4096
 * workgroups; escapes beyond a workgroup's share are resolved in the
 * streaming pass, with the same result, more slowly).  Asynchronous on
 * `stream`.
 * Errors: ROIX_EINVAL (NULL ctx/out/d_info/info pointers, bad dims or dtype,
 * misaligned buffers, negative capacity), ROIX_ENOMEM (arena under 32 KB),
 * ROIX_EDEVICE. */
typedef struct {
    int32_t status;
    int32_t pad;
    uint64_t n_codes;
} roix_section_info; /* 16 bytes */
roix_status roix_section(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims,
                         const roix_fused_out* out, uint8_t* d_section, int64_t section_cap,
                         roix_section_info* d_info, void* stream);

/* Absolute error-bounded quantisation of an 8-bit pixel sequence, the
 * paper's own algorithm (Sec. 4.2.3): a group grows pixel by
 * pixel while the intervals [D - E, D + E] of its pixels intersect, and
 * every pixel of the group is written as the floor of the midpoint of that
 * intersection, floor((min + max) / 2), clipped to 0..255.  The pixels are
 * integers, so the tolerance taken is floor(e_abs), which keeps
 * |Q - D| <= e_abs for every pixel (with a fractional tolerance the floored
 * midpoint could miss the bound).  The result is the sequential scan's,
 * bit for bit.
 *   d_pixels  m uint8 pixels (e.g. the 8-bit normalised pixel section of
 *             Sec. 4.1.2), 16-byte aligned
 *   d_q       m uint8 outputs, 16-byte aligned, not overlapping d_pixels
 *             (the output is written while later passes still read pixels)
 *   d_info    device: status, n_groups (the number of groups), rounds (the
 *             fix-up rounds that ran) and finisher_chunks (chunks settled
 *             by the sequential pass; see below)
 * The context's arena holds roix_abs_quantize_scratch_bytes(m) bytes of
 * per-chunk state (about 49 bytes per 256 pixels) while the call runs.
 * Sequences are cut into chunks of 256 pixels scanned in parallel from a
 * guessed start and corrected in up to 4 rounds; chunks whose groups still
 * depend on an earlier chunk after that (group chains that never meet, as
 * on long exact ramps) are settled by a single-wave sequential pass, which
 * is correct but slow.  Asynchronous on `stream`.
 * Errors: ROIX_EINVAL (NULL ctx/d_info, NULL or misaligned buffers for
 * m > 0, m < 0, e_abs negative or NaN, overlapping buffers), ROIX_ENOMEM (arena
 * too small), ROIX_EDEVICE. */
typedef struct {
    int32_t status;
    int32_t rounds;
    uint64_t n_groups;
    uint64_t finisher_chunks;
    uint64_t pad;
} roix_absq_info; /* 32 bytes */
size_t roix_abs_quantize_scratch_bytes(int64_t m);
roix_status roix_abs_quantize(roix_ctx* ctx, const uint8_t* d_pixels, int64_t m, double e_abs, uint8_t* d_q,
                              roix_absq_info* d_info, void* stream);

/* Lossless Huffman stage for a byte sequence (the packed code stream, or the
 * output of roix_abs_quantize): Huffman coding, which Sec. 1 lists among the
 * lossless coders a ROI representation can be handed to.
 * Code lengths follow Huffman's construction over the 256 byte counts, with
 * equal weights ordered by (count, byte value) for leaves and by creation
 * for merged nodes, a leaf first on a tie; a single used byte gets length 1.
 * Codes are canonical (within a length increasing with the byte value; the
 * first code of a length follows the last of the length before, shifted
 * left).  Format: blocks of 4096 input bytes; block b starts at 32-bit word
 * block_off[b] of the payload, its codes written one after another from the
 * most significant bit of each word down, zero bits to the end of its last
 * word; block_off[nblocks] is the payload length in words.
 * Sub-block index (optional): every block is cut into 16 sub-blocks of 256
 * input bytes and sub_bits[16 b + k] holds the code bits of sub-block k of
 * block b (0 past the input's end; at most 8192).  Sub-blocks follow each
 * other in the payload with no padding, so the payload is the same with or
 * without the index; sub-block k starts at bit sub_bits[16 b] + ... +
 * sub_bits[16 b + k - 1] of its block, which lets a decoder start at every
 * sub-block at once.
 * The compressed form is lengths (256 bytes) + block_off (8 bytes per
 * block + 8) + payload (4 bytes per word), + the index (32 bytes per block)
 * when one is written: info.compressed_bytes.
 *   d_in          n bytes, 16-byte aligned
 *   d_lengths     out: 256 code lengths (0 = byte unused)
 *   d_block_off   out: nblocks + 1 offsets, nblocks = ceil(n / 4096)
 *   d_sub_bits    out: 16 nblocks sub-block bit counts (2-byte aligned), or
 *                 NULL for no index
 *   d_payload     out: payload_cap_words words; at most 32 bits per input
 *                 byte, so 4096 words per block always suffice
 *   d_info        device: status, max_len, n, n_blocks, payload_words,
 *                 compressed_bytes
 * info.status: ROIX_ERANGE when a code length would exceed 32 bits (counts
 * growing like the Fibonacci numbers over more than 33 bytes; the payload is
 * then unspecified), ROIX_ETRUNC when the payload exceeds payload_cap_words
 * (the offsets and sizes are still complete; blocks that do not fit are not
 * written).  The context's arena holds about 20 KB of state and tables while
 * the call runs.
 * Errors: ROIX_EINVAL (NULL or misaligned buffers, n outside 0..2^40,
 * negative capacity), ROIX_ENOMEM (arena too small), ROIX_EDEVICE. */
typedef struct {
    int32_t status;
    int32_t max_len;
    uint64_t n;
    uint64_t n_blocks;
    uint64_t payload_words;
    uint64_t compressed_bytes;
    uint64_t pad[3];
} roix_huff_info; /* 64 bytes */
roix_status roix_huff_encode(roix_ctx* ctx, const uint8_t* d_in, int64_t n, uint8_t* d_lengths,
                             uint64_t* d_block_off, uint16_t* d_sub_bits, uint32_t* d_payload,
                             int64_t payload_cap_words, roix_huff_info* d_info, void* stream);

/* Decode n bytes from the format of roix_huff_encode into d_out (16-byte
 * aligned).  With the sub-block index (d_sub_bits, 16 nblocks entries) a
 * lane decodes a 256-byte sub-block from the start the index gives (16 lanes
 * per block); without it (NULL) a lane decodes a whole block.  info.status
 * is ROIX_EINVAL when the lengths are no prefix code (a length above 32,
 * Kraft sum above 1, none used for n > 0), the offsets do not start at 0,
 * decrease or pass payload_words, a block's (sub-block's) bits end or match
 * no code before its bytes are complete, or, with the index, a sub-block's
 * codes do not take exactly its stated bits or a block's stated bits exceed
 * its words; d_out is then unspecified.  Errors as roix_huff_encode. */
roix_status roix_huff_decode(roix_ctx* ctx, const uint8_t* d_lengths, const uint64_t* d_block_off,
                             const uint16_t* d_sub_bits, const uint32_t* d_payload, int64_t payload_words, int64_t n,
                             uint8_t* d_out, roix_huff_info* d_info, void* stream);

/* One volume of a batch: input, shape, bound, criterion and the caller's
 * output buffers (as for roix_fused).  Each volume's outputs sit in its own
 * descriptor, so one array describes the whole batch. */
typedef struct {
    const void* d_in;
    int32_t dtype; /* roix_dtype */
    int32_t pad;
    roix_dims dims;
    roix_eb eb;
    roix_criterion crit;
    roix_fused_out out;
} roix_volume_desc;

/* Batched form: every volume of `vols` through the fused path, with output
 * identical to n separate roix_fused calls, in one launch per stage for all
 * the volumes.  Each volume's launch sequence is that of roix_fused on its
 * own part of the arena (the voxel-proportional passes on its share of the
 * grid); the sequences are merged so that each kernel runs once for every
 * volume that needs it next, each workgroup finding its volume in a device
 * table of arguments.  Volumes whose worst-case layouts do not all fit the
 * arena at once run in consecutive groups.  The merged sequence (about 30
 * launches, whatever the number of volumes) is recorded once and kept while
 * the batch's structure -- volume shapes, flows, grids, parameters -- is the
 * same; buffer addresses may change from call to call.  It is issued as
 * direct launches, or with batch_graph = 1 captured into a HIP graph and
 * replayed.  Asynchronous on `stream`; the argument tables are
 * copied from pinned host memory the context keeps (allocated, or grown, on
 * the first batch that needs it).  Errors: ROIX_EINVAL (NULL ctx/vols, any
 * invalid descriptor), ROIX_ENOMEM (a volume does not fit the arena even
 * alone), ROIX_EDEVICE. */
roix_status roix_fused_batch(roix_ctx* ctx, int32_t n, const roix_volume_desc* vols, void* stream);

/* Launch parameters of a context (the autotuner's knobs):
 *   "grid_stream"    workgroups of the grid-stride streaming kernels
 *   "grid_read"      workgroups of the read-only range kernel
 *   "grid_emit"      workgroups of the code-emit kernels
 *   "grid_mask"      workgroups of the mask-word and run kernels
 *   "seg_grid"       workgroups of the component-labelling kernels
 *   "stats_grid"     workgroups of the component-statistics kernel
 *   "seg_runs"       runs labelled together in one workgroup's local memory
 *                    (a multiple of 256 up to 16384; 0 = spread the runs over
 *                    seg_grid workgroups, at least 2048 each)
 *   "batch_group"    volumes per launch group of roix_fused_batch (0 = as
 *                    many as the arena holds; 1 = one volume at a time)
 *   "batch_lanes"    1..4 concurrent launch sequences of roix_fused_batch
 *                    (default 2): volume i goes to lane i mod lanes, each lane
 *                    on its own part of the arena; lane 0 runs on the caller's
 *                    stream, the others on streams of the context that start
 *                    after the call's earlier work on the caller's stream and
 *                    that stream waits for before its next work.  One lane
 *                    when batch_graph is 1 or a volume does not fit a part.
 *   "batch_graph"    1 = capture/replay batches as a HIP graph, 0 = launch
 *                    directly (default: a batch is about 30 launches, and
 *                    their direct launch costs less host time than the
 *                    graph's launch)
 *   "batch_fused16_min_voxels"  as fused16_min_voxels, for the volumes of a
 *                    batch (default 2^26: below it the one-pass flow's
 *                    per-workgroup class tables outweigh its saved read)
 *   "fused16_min_voxels"  smallest float32 volume (voxels) that the fused path
 *                    quantises in one pass with the range, writing a 16-bit
 *                    code proxy, when the bound is absolute, rows hold a
 *                    multiple of 4 voxels and start 16-byte aligned, and the
 *                    arena has room (default 2^22; 0..2^40)
 *   "compute_units"  (get only) the device's compute units
 * None of them changes any output.  Errors: ROIX_EINVAL (unknown name or
 * value out of range). */
roix_status roix_ctx_set_param(roix_ctx* ctx, const char* name, int64_t value);
roix_status roix_ctx_get_param(roix_ctx* ctx, const char* name, int64_t* value);

/* Autotuner of the launch parameters above, on the caller's own volume.
 * Runs roix_fused with the given arguments and tunes grid_stream,
 * grid_read, grid_mask, grid_emit, seg_grid, stats_grid and then seg_runs by
 * coordinate descent: for each knob in that order, each candidate (4, 8, 16
 * x CUs; 1, 2, 4; 16, 32, 64; 2, 4, 8; 1, 2, 4; 1, 2, 4 x CUs; seg_runs 0,
 * 1024, 2048, 4096) is timed as the median of `reps` runs (HIP events on
 * `stream`) with the other knobs held, and the fastest is kept on the
 * context.  Every candidate's outputs must equal the first run's (the info
 * structs byte for byte, position-weighted checksums of the row table, code
 * stream, outliers and component table): a difference is a defect and
 * returns ROIX_EDEVICE with the knob restored.
 * cache_path (may be NULL): a text file of tuned values keyed by the
 * device's architecture, dtype, bound mode, connectivity, threshold mode and
 * the power-of-two buckets of nx, ny, nz.  On a hit the values are applied
 * without timing (from_cache = 1); after tuning the line is appended.
 * Synchronous: it waits for its runs.  The outputs hold the last run's
 * results (those of every candidate).  res->status is the outputs'
 * extraction status when it is not OK (nothing is tuned then), or
 * ROIX_EDEVICE on a difference.  It allocates 32 bytes of device memory for
 * the checksums while it runs.
 * Errors: those of roix_fused; ROIX_EINVAL (NULL res, reps outside 1..100,
 * NULL info pointers in out), ROIX_EDEVICE. */
typedef struct {
    int32_t status;
    int32_t n_timed;      /* fused runs timed */
    int32_t from_cache;
    int32_t pad;
    double default_ms;    /* median with the context's parameters before tuning (-1 from the cache) */
    double best_ms;       /* median with the chosen parameters (-1 from the cache) */
    int64_t params[7];    /* grid_stream, grid_read, grid_mask, grid_emit, seg_grid, stats_grid, seg_runs */
} roix_tune_result;       /* 88 bytes */
roix_status roix_autotune(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                          const roix_criterion* crit, const roix_fused_out* out, int32_t reps,
                          const char* cache_path, roix_tune_result* res, void* stream);

/* Per-stage GPU timing.  When enabled, every kernel of the fused, staged
 * and batched paths is bracketed by HIP events on its stream;
 * roix_ctx_read_timing synchronises those events and returns, per stage,
 * the accumulated milliseconds and launch counts since the last read
 * (arrays of roix_stage_count() entries), then clears them. */
int roix_stage_count(void);
const char* roix_stage_name(int stage);
roix_status roix_ctx_set_timing(roix_ctx* ctx, int enable);
roix_status roix_ctx_read_timing(roix_ctx* ctx, double* ms, int64_t* launches);

/* ------------------------------------------------------------------ served
 *
 * Served form: volumes arrive as consecutive z-slabs (a detector streaming
 * projections, or a reconstruction written slab by slab) and are reduced
 * while they arrive.  A server owns an HBM pool of `hbm_budget_bytes`
 * (allocated once at roix_server_create), a copy stream and a compute
 * stream of its own.
 *
 * A volume is admitted at roix_volume_open when its resident footprint
 * (roix_server_volume_bytes) fits the free part of the pool; otherwise the
 * call returns ROIX_EBUSY and nothing is kept (the caller retries after a
 * volume has closed).  Every slab is copied (host or device memory) into
 * the volume's resident buffer on the copy stream.
 *
 * With an absolute bound and a FIXED threshold the mask of a voxel is known
 * when its slab arrives (the readings of Sec. 4.1.3-4.1.4 for a fixed
 * threshold: object = q(x) > q(T)), so each slab is reduced at once: value
 * range, mask, runs, and the connected components of the slab's runs,
 * united with the runs of the earlier slabs that stay resident on the
 * device.  The keep rule, the spans and the code stream depend on the whole
 * volume (LARGEST, qmin), so they run at roix_volume_close.  Volumes with an
 * OTSU threshold or a REL bound only collect slabs and run the whole path at
 * close.  Either way the outputs equal roix_fused on the assembled volume
 * with the same arguments.
 *
 * A uint16 volume with an absolute bound and a FIXED threshold whose codes
 * cannot span more than 2^15 values (rint(65535 / (2 eb32)) < 2^15, i.e. eb
 * of about 1 or more) is not kept whole: each slab is staged (at most
 * "slab_planes" planes at a time), and only each row's extent -- from its
 * first to its last mask voxel, where every span of the row must lie -- is
 * kept, in a store of "store_permille" per mille of the volume's voxels;
 * counts of the code classes q mod 2^15 stand in for the histogram, which
 * close rebuilds once the range is known (Sec. 4.1.2).  A volume whose
 * extents outgrow the store fails with ROIX_ENOMEM in its infos at close.
 *
 * Requests complete asynchronously; roix_wait returns their host-clock
 * times.  Slab latency = completion - submission (copy and compute,
 * including the wait behind earlier requests).  All calls on one server
 * must come from one host thread. */
typedef struct roix_server roix_server;

typedef enum { ROIX_REQ_SLAB = 0, ROIX_REQ_CLOSE = 1 } roix_req_kind;

typedef struct {
    int32_t status;    /* ROIX_OK, or the device error of the request */
    int32_t kind;      /* roix_req_kind */
    int64_t vol_id;
    double submit_ms;  /* host steady clock, ms since roix_server_create */
    double done_ms;    /* completion on the device, same clock */
    double latency_ms; /* done_ms - submit_ms */
} roix_req_result;

typedef struct {
    int64_t volumes_admitted, volumes_refused, volumes_open;
    int64_t slabs_done, closes_done;
    int64_t bytes_in;            /* slab bytes accepted */
    uint64_t budget_bytes, bytes_in_use;
    double slab_p50_ms, slab_p99_ms, slab_max_ms; /* over completed slabs */
    double close_p50_ms, close_p99_ms;
} roix_server_stats_t;

/* Server on ctx's device with an HBM pool of hbm_budget_bytes.  The server
 * does not use ctx's arena; ctx must outlive the server.  Errors:
 * ROIX_EINVAL (NULL ctx/out, zero budget), ROIX_ENOMEM (the pool cannot be
 * allocated), ROIX_EDEVICE. */
roix_status roix_server_create(roix_ctx* ctx, size_t hbm_budget_bytes, roix_server** out);
/* Waits for all work, then frees the pool, streams and events. */
roix_status roix_server_destroy(roix_server* srv);

/* Pool bytes a volume holds while open on this server: its input
 * (N * voxel bytes) plus the labelling state (no proxy for incremental
 * volumes) with run arrays for runs_per_row runs per row on average (a
 * volume with more foreground runs fails with ROIX_ENOMEM in its infos at
 * close); for a volume kept as row extents, its stage, store, row tables,
 * code-class counts and run arrays instead of the input.  0 for invalid
 * arguments. */
size_t roix_server_volume_bytes(const roix_server* srv, roix_dims dims, roix_dtype dtype, roix_eb eb,
                                const roix_criterion* crit);

/* Server parameters (each applies to volumes opened from now on):
 *   "runs_per_row"  run-array capacity, as an average number of foreground
 *                   runs per row (default 32, capped at the worst case of
 *                   ceil(nx/2))
 *   "slab_planes"   planes a volume kept as row extents stages at once
 *                   (1..4096, default 32; larger slabs are staged in turn)
 *   "store_permille" store of a volume kept as row extents, per mille of its
 *                   voxels (1..1000, default 500)
 * Errors: ROIX_EINVAL (unknown name or value out of range). */
roix_status roix_server_set_param(roix_server* srv, const char* name, int64_t value);

/* Admit a volume.  `final_out` (copied; its buffers must stay valid until the
 * close request completes) receives the outputs at close.  Errors:
 * ROIX_EINVAL (arguments, as roix_fused), ROIX_EBUSY (the pool has no room
 * now). */
roix_status roix_volume_open(roix_server* srv, roix_dims dims, roix_dtype dtype, roix_eb eb,
                             const roix_criterion* crit, const roix_fused_out* final_out, int64_t* vol_id);

/* Submit planes [z0, z0 + nz_slab) of volume vol_id from `ptr` (host memory
 * when ptr_is_device == 0 -- pinned memory gives an asynchronous copy --
 * else device memory), C-contiguous [nz_slab][ny][nx].  The memory must stay
 * untouched until the request completes.  Slabs must come in order: z0 must
 * equal the end of the previous slab.  Errors: ROIX_EINVAL (unknown volume,
 * NULL ptr, nz_slab < 1, z0 + nz_slab > nz), ROIX_ESEQ (z0 out of order or
 * repeated, volume already closed). */
roix_status roix_slab_submit(roix_server* srv, int64_t vol_id, int64_t z0, int64_t nz_slab, const void* ptr,
                             int ptr_is_device, int64_t* req_id);

/* Enqueue the end of volume vol_id: the remaining stages and the outputs.
 * The volume's pool memory is released when the request completes.  The
 * close is a request like a slab's: *req_id (nullable) is what roix_wait
 * takes to learn when the outputs are complete and how long the close took.
 * Errors: ROIX_EINVAL (unknown volume), ROIX_ESEQ (slabs missing, or already
 * closed). */
roix_status roix_volume_close(roix_server* srv, int64_t vol_id, int64_t* req_id);

/* Drop a volume: no outputs; its memory is released once its enqueued work
 * has finished.  Errors: ROIX_EINVAL (unknown volume), ROIX_ESEQ (already
 * closed or aborted). */
roix_status roix_volume_abort(roix_server* srv, int64_t vol_id);

/* Wait up to timeout_ms (< 0: forever) for a request.  ROIX_OK with *res
 * filled (the request is then forgotten), ROIX_EBUSY if it has not
 * completed in time, ROIX_EINVAL for an unknown id. */
roix_status roix_wait(roix_server* srv, int64_t req_id, int64_t timeout_ms, roix_req_result* res);

roix_status roix_server_stats(roix_server* srv, roix_server_stats_t* out);

const char* roix_status_string(roix_status st);

/* sizeof of a public struct by name ("roix_quant_info", "roix_seg_info",
 * "roix_extract_info", "roix_component", "roix_row", "roix_fused_out",
 * "roix_criterion", "roix_eb", "roix_dims", "roix_volume_desc",
 * "roix_req_result", "roix_server_stats_t", "roix_decode_info"), 0 if unknown: lets bindings
 * check their mirrors of this header. */
size_t roix_sizeof(const char* type_name);

#ifdef __cplusplus
}
#endif

#endif /* ROIX_H */
