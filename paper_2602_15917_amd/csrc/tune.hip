// tune.hip - the autotuner of a context's launch parameters.
//
// roix_autotune runs the fused path on the caller's own volume and picks the
// launch parameters by coordinate descent: one knob at a time, every
// candidate value timed (median of `reps` runs, HIP events on the caller's
// stream) with the others held, the fastest kept.  No launch parameter may
// change an output, so every candidate's outputs are checked against the
// first run's: the three info structs byte for byte, and position-weighted
// 64-bit checksums of the row table, the code stream, the outliers and the
// component table.  A difference is a defect and fails the call.  The
// result can be kept in a plain-text cache keyed by the device's
// architecture, dtype, bound mode, connectivity, threshold mode and the
// power-of-two buckets of the dimensions, so that later contexts take the
// tuned values without timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"

namespace roix {

// sum over the buffer's 32-bit words of word * (2 i + 1), mod 2^64: any
// change of a word or of the order changes it (with overwhelming odds)
__global__ __launch_bounds__(256) void k_checksum(const uint8_t* __restrict__ p, unsigned long long nbytes,
                                                  unsigned long long* out) {
    const unsigned long long nw = nbytes / 4;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
    unsigned long long acc = 0ull;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride)
        acc += (unsigned long long)w[i] * (2ull * i + 1ull);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (unsigned long long b = nw * 4; b < nbytes; ++b) acc += (unsigned long long)p[b] * (2ull * b + 7ull);
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) atomicAdd(out, acc);
}

__global__ void k_checksum_clear(unsigned long long* s) {
    if (threadIdx.x < 4) s[threadIdx.x] = 0ull;
}

namespace {

struct Signature {
    roix_quant_info q;
    roix_seg_info s;
    roix_extract_info e;
    unsigned long long sums[4];
    bool operator==(const Signature& o) const {
        return memcmp(&q, &o.q, sizeof q) == 0 && memcmp(&s, &o.s, sizeof s) == 0 &&
               memcmp(&e, &o.e, sizeof e) == 0 && memcmp(sums, o.sums, sizeof sums) == 0;
    }
};

struct Tuner {
    roix_ctx* ctx;
    const void* in;
    roix_dtype dt;
    roix_dims dims;
    roix_eb eb;
    const roix_criterion* crit;
    const roix_fused_out* out;
    hipStream_t st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    unsigned long long* dsum = nullptr;  // 4 device accumulators
    int timed = 0;

    roix_status run(double* ms) {
        if (hipEventRecord(e0, st) != hipSuccess) return ROIX_EDEVICE;
        roix_status rc = roix_fused(ctx, in, dt, dims, eb, crit, out, st);
        if (rc != ROIX_OK) return rc;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ROIX_EDEVICE;
        float f = 0.0f;
        if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return ROIX_EDEVICE;
        *ms = f;
        ++timed;
        return ROIX_OK;
    }

    roix_status median(int reps, double* ms) {
        std::vector<double> t((size_t)reps);
        for (int i = 0; i < reps; ++i) {
            roix_status rc = run(&t[(size_t)i]);
            if (rc != ROIX_OK) return rc;
        }
        std::sort(t.begin(), t.end());
        *ms = t[(size_t)reps / 2];
        return ROIX_OK;
    }

    roix_status signature(Signature* sig) {
        if (hipMemcpyAsync(&sig->q, out->d_qinfo, sizeof sig->q, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&sig->s, out->d_sinfo, sizeof sig->s, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&sig->e, out->d_einfo, sizeof sig->e, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return ROIX_EDEVICE;
        const unsigned long long nrows = std::min<unsigned long long>(sig->e.n_rows, (unsigned long long)out->rows_cap);
        const unsigned long long nsb =
            std::min<unsigned long long>(sig->e.stream_bytes, (unsigned long long)out->stream_cap_bytes);
        const unsigned long long nout =
            std::min<unsigned long long>(sig->e.n_outliers, (unsigned long long)out->outliers_cap);
        const unsigned long long ncomp =
            std::min<unsigned long long>(sig->s.n_components, (unsigned long long)out->comps_cap);
        const struct {
            const void* p;
            unsigned long long n;
        } bufs[4] = {{out->d_rows, nrows * sizeof(roix_row)},
                     {out->d_stream, nsb},
                     {out->d_outliers, nout * 4ull},
                     {out->d_comps, ncomp * sizeof(roix_component)}};
        hipLaunchKernelGGL(k_checksum_clear, dim3(1), dim3(4), 0, st, dsum);
        for (int i = 0; i < 4; ++i) {
            if (!bufs[i].p || bufs[i].n == 0) continue;
            const unsigned long long g = (bufs[i].n / 4 + 255) / 256;
            const int grid = (int)(g < 1 ? 1 : g < 4096 ? g : 4096);
            hipLaunchKernelGGL(k_checksum, dim3(grid), dim3(256), 0, st, (const uint8_t*)bufs[i].p, bufs[i].n,
                               dsum + i);
        }
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sig->sums, dsum, sizeof sig->sums, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return ROIX_EDEVICE;
        return ROIX_OK;
    }
};

int64_t bucket(int64_t v) {
    int64_t b = 1;
    while (b < v) b <<= 1;
    return b;
}

std::string cache_key(roix_ctx* ctx, roix_dtype dt, roix_dims d, roix_eb eb, const roix_criterion* c) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[256];
    snprintf(buf, sizeof buf, "%s/dt%d/eb%d/conn%d/thr%d/%lldx%lldx%lld", arch.c_str(), (int)dt, (int)eb.mode,
             (int)c->connectivity, (int)c->thr, (long long)bucket(d.nx), (long long)bucket(d.ny),
             (long long)bucket(d.nz));
    return buf;
}

}  // namespace

}  // namespace roix

using namespace roix;

namespace {
// the knobs in the order they are tuned, with candidate multiples of the CU count
struct Knob {
    const char* name;
    int mult[4];
};
const Knob kKnobs[] = {
    {"grid_stream", {4, 8, 16, 0}}, {"grid_read", {1, 2, 4, 0}},    {"grid_mask", {16, 32, 64, 0}},
    {"grid_emit", {2, 4, 8, 0}},    {"seg_grid", {1, 2, 4, 0}},     {"stats_grid", {1, 2, 4, 0}},
};
const int64_t kSegRuns[] = {0, 1024, 2048, 4096};
constexpr int kNumParams = 7;  // the six knobs above, then seg_runs
const char* param_name(int i) { return i < 6 ? kKnobs[i].name : "seg_runs"; }
}  // namespace

extern "C" {

roix_status roix_autotune(roix_ctx* ctx, const void* d_in, roix_dtype dtype, roix_dims dims, roix_eb eb,
                          const roix_criterion* crit, const roix_fused_out* out, int32_t reps,
                          const char* cache_path, roix_tune_result* res, void* stream) {
    if (!ctx || !res || !out || !crit || reps < 1 || reps > 100) return ROIX_EINVAL;
    if (!out->d_qinfo || !out->d_sinfo || !out->d_einfo) return ROIX_EINVAL;
    memset(res, 0, sizeof *res);
    const std::string key = cache_key(ctx, dtype, dims, eb, crit);
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            char line[1024];
            bool hit = false;
            while (!hit && fgets(line, sizeof line, f)) {
                char k[512];
                long long v[kNumParams];
                if (sscanf(line, "%511s %lld %lld %lld %lld %lld %lld %lld", k, &v[0], &v[1], &v[2], &v[3], &v[4],
                           &v[5], &v[6]) == 8 &&
                    key == k) {
                    hit = true;
                    for (int i = 0; i < kNumParams; ++i)
                        if (roix_ctx_set_param(ctx, param_name(i), v[i]) != ROIX_OK) hit = false;
                    for (int i = 0; i < kNumParams; ++i) res->params[i] = v[i];
                }
            }
            fclose(f);
            if (hit) {
                res->from_cache = 1;
                res->default_ms = res->best_ms = -1.0;
                return ROIX_OK;
            }
        }
    }
    Tuner t;
    t.ctx = ctx;
    t.in = d_in;
    t.dt = dtype;
    t.dims = dims;
    t.eb = eb;
    t.crit = crit;
    t.out = out;
    t.st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess || hipEventCreate(&t.e0) != hipSuccess ||
        hipEventCreate(&t.e1) != hipSuccess || hipMalloc(&t.dsum, 4 * sizeof(unsigned long long)) != hipSuccess) {
        if (t.e0) hipEventDestroy(t.e0);
        if (t.e1) hipEventDestroy(t.e1);
        return ROIX_EDEVICE;
    }
    auto finish = [&](roix_status rc) {
        hipEventDestroy(t.e0);
        hipEventDestroy(t.e1);
        hipFree(t.dsum);
        res->n_timed = t.timed;
        return rc;
    };
    double ms = 0.0;
    roix_status rc = t.run(&ms);  // warm-up (and argument check)
    if (rc != ROIX_OK) return finish(rc);
    Signature base;
    if ((rc = t.signature(&base)) != ROIX_OK) return finish(rc);
    if (base.e.status != ROIX_OK) {  // outputs the caller's buffers cannot hold, or bad data
        res->status = base.e.status;
        return finish(ROIX_OK);
    }
    if ((rc = t.median(reps, &ms)) != ROIX_OK) return finish(rc);
    res->default_ms = ms;
    double best = ms;
    for (int k = 0; k < kNumParams; ++k) {
        const char* name = param_name(k);
        int64_t cur = 0;
        roix_ctx_get_param(ctx, name, &cur);
        std::vector<int64_t> cand;
        if (k < 6) {
            for (int m : kKnobs[k].mult)
                if (m > 0) cand.push_back((int64_t)m * ctx->cus);
        } else {
            cand.assign(std::begin(kSegRuns), std::end(kSegRuns));
        }
        int64_t keep = cur;
        for (int64_t v : cand) {
            if (v == cur || roix_ctx_set_param(ctx, name, v) != ROIX_OK) continue;
            double m = 0.0;
            if ((rc = t.median(reps, &m)) != ROIX_OK) {
                roix_ctx_set_param(ctx, name, cur);
                return finish(rc);
            }
            Signature sig;
            if ((rc = t.signature(&sig)) != ROIX_OK) return finish(rc);
            if (!(sig == base)) {  // a launch parameter changed an output: a defect
                roix_ctx_set_param(ctx, name, cur);
                res->status = ROIX_EDEVICE;
                return finish(ROIX_EDEVICE);
            }
            if (m < best) {
                best = m;
                keep = v;
            }
        }
        roix_ctx_set_param(ctx, name, keep);
        res->params[k] = keep;
    }
    res->best_ms = best;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "a")) {
            fprintf(f, "%s", key.c_str());
            for (int i = 0; i < kNumParams; ++i) fprintf(f, " %lld", (long long)res->params[i]);
            fprintf(f, "\n");
            fclose(f);
        }
    }
    return finish(ROIX_OK);
}

}  // extern "C"
