// libxeng.so: host side of the X-engine C ABI declared in include/xeng.h.
//
// Owns the per-subarray int32 accumulators (already in the packed output
// layout, so a dump is a plain copy), checks the exactness bounds before any
// launch, splits each call into segments of at most SEG_T samples and
// launches the tile kernels on the context's stream.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/xeng.h"
#include "xcorr_i8.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(XENG_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                           \
    } while (0)

struct Sub {
    xeng_subarray cfg{};
    int32_t *d_acc = nullptr;  // [F][tri][2]
    int64_t tri = 0;
    int64_t since_dump = 0;    // samples accumulated since the last reset
    int64_t max_dump = 0;      // exactness bound on since_dump
    bool acc_zero = true;      // accumulator logically zero (next launch overwrites)
    int wt = 4;                // wave tile edge in 16-row sub-blocks
    int bt = 128;              // workgroup tile edge
    int n_tiles = 0;
};

} // namespace

struct xeng_ctx {
    std::vector<Sub> subs;
    hipStream_t stream = nullptr;
    int device = 0;
};

namespace {

using KernelFn = void (*)(xeng::TileArgs);

template <int IN_BITS, bool AL>
KernelFn pick_wt(int wt)
{
    if (wt == 1) return xeng::xcorr_i8_kernel<IN_BITS, 1, AL>;
    if (wt == 2) return xeng::xcorr_i8_kernel<IN_BITS, 2, AL>;
    return xeng::xcorr_i8_kernel<IN_BITS, 4, AL>;
}

constexpr int DMA_NBUF = 4; // LDS ring depth of the direct-staging kernel

// 4-bit input whose rows split into whole 16-byte chunks takes the
// direct-staging kernel; everything else the register-staging kernel (whole
// dword loads when a dword holds whole inputs, else byte loads).
bool use_dma(int in_bits, int n_inputs) { return in_bits == 4 && n_inputs % 16 == 0; }

KernelFn pick_kernel(int in_bits, int wt, int n_inputs)
{
    if (use_dma(in_bits, n_inputs)) {
        if (wt == 1) return xeng::xcorr4_dma_kernel<1, DMA_NBUF>;
        if (wt == 2) return xeng::xcorr4_dma_kernel<2, DMA_NBUF>;
        return xeng::xcorr4_dma_kernel<4, DMA_NBUF>;
    }
    if (in_bits == 4)
        return (n_inputs % 4 == 0) ? pick_wt<4, true>(wt) : pick_wt<4, false>(wt);
    return (n_inputs % 2 == 0) ? pick_wt<8, true>(wt) : pick_wt<8, false>(wt);
}

// Tile edge per input count: the smallest workgroup tile that covers N, up
// to 128 inputs per side.
int choose_wt(int n_inputs)
{
    if (n_inputs <= 32) return 1;
    if (n_inputs <= 64) return 2;
    return 4;
}

int validate(const xeng_subarray &s, int idx)
{
    if (s.n_inputs < 1 || s.n_inputs > 65536)
        return fail(XENG_EINVAL, "subarray %d: n_inputs %d out of [1, 65536]", idx, s.n_inputs);
    if (s.n_chans < 1)
        return fail(XENG_EINVAL, "subarray %d: n_chans %d < 1", idx, s.n_chans);
    if (s.n_time < 1)
        return fail(XENG_EINVAL, "subarray %d: n_time %d < 1", idx, s.n_time);
    if (s.in_bits != 4 && s.in_bits != 8)
        return fail(XENG_EINVAL, "subarray %d: in_bits %d is not 4 or 8", idx, s.in_bits);
    if (s.engine != XENG_ENGINE_I8 && s.engine != XENG_ENGINE_FP8)
        return fail(XENG_EINVAL, "subarray %d: unknown engine %d", idx, s.engine);
    if (s.engine == XENG_ENGINE_FP8)
        return fail(XENG_EINVAL, "subarray %d: the FP8 engine is not available in this build", idx);
    if (s.engine == XENG_ENGINE_FP8 && s.in_bits != 4)
        return fail(XENG_EINVAL, "subarray %d: the FP8 engine takes 4-bit input only", idx);
    if (s.engine == XENG_ENGINE_FP8 && s.n_time > XENG_MAX_CALL_SAMPLES_FP8)
        return fail(XENG_EINVAL, "subarray %d: n_time %d above the FP8 per-call limit %lld", idx,
                    s.n_time, (long long)XENG_MAX_CALL_SAMPLES_FP8);
    const int64_t tri = (int64_t)s.n_inputs * (s.n_inputs + 1) / 2;
    const int64_t nb = (s.n_inputs + 127) / 128;
    if (tri * (int64_t)s.n_chans * 2 > ((int64_t)1 << 40) || nb * (nb + 1) / 2 * s.n_chans > INT32_MAX)
        return fail(XENG_EINVAL, "subarray %d: output too large", idx);
    // one LDS stage of the tile kernel spans TK time rows of the whole
    // [F][N] plane; its byte offsets must fit the 32-bit buffer offsets
    if ((int64_t)s.n_chans * s.n_inputs * (s.in_bits / 4) * xeng::TK >= ((int64_t)1 << 31))
        return fail(XENG_EINVAL, "subarray %d: n_chans * n_inputs too large for one stream", idx);
    const int64_t bound = s.in_bits == 4 ? XENG_MAX_DUMP_SAMPLES_4BIT : XENG_MAX_DUMP_SAMPLES_8BIT;
    if (s.n_time > bound)
        return fail(XENG_EINVAL, "subarray %d: n_time %d above the dump limit %lld", idx, s.n_time,
                    (long long)bound);
    return XENG_OK;
}

int zero_device(int32_t *p, size_t n_words, hipStream_t st)
{
    const size_t n16 = n_words / 4, ntail = n_words % 4;
    int blocks = (int)((n16 + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(xeng::fill_zero_kernel, dim3(blocks), dim3(256), 0, st, (int4 *)p, n16,
                       p + n16 * 4, ntail);
    HIP_TRY(hipGetLastError());
    return XENG_OK;
}

int launch_sub(Sub &s, const void *d_samples, hipStream_t st)
{
    const xeng_subarray &c = s.cfg;
    KernelFn fn = pick_kernel(c.in_bits, s.wt, c.n_inputs);
    for (int64_t t0 = 0; t0 < c.n_time; t0 += xeng::SEG_T) {
        xeng::TileArgs a;
        a.samples = (const uint8_t *)d_samples;
        a.vis = s.d_acc;
        a.t_begin = t0;
        a.t_count = (int32_t)((c.n_time - t0) < xeng::SEG_T ? (c.n_time - t0) : xeng::SEG_T);
        a.n_chans = c.n_chans;
        a.n_inputs = c.n_inputs;
        a.n_tiles = s.n_tiles;
        a.n_work = s.n_tiles * c.n_chans;
        a.accumulate = s.acc_zero ? 0 : 1;
        hipLaunchKernelGGL(fn, dim3(a.n_work), dim3(xeng::WG_THREADS), 0, st, a);
        HIP_TRY(hipGetLastError());
        s.acc_zero = false;
    }
    return XENG_OK;
}

} // namespace

extern "C" {

const char *xeng_strerror(int code)
{
    switch (code) {
    case XENG_OK: return "ok";
    case XENG_EINVAL: return "invalid argument";
    case XENG_ERANGE: return "exactness bound exceeded";
    case XENG_ENOMEM: return "out of device memory";
    case XENG_EHIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

const char *xeng_last_error(void) { return g_last_error.c_str(); }

int xeng_create(const xeng_subarray *subs, int n_subs, void *hip_stream, xeng_ctx **out)
{
    if (!out) return fail(XENG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!subs) return fail(XENG_EINVAL, "subs is NULL");
    if (n_subs < 1 || n_subs > 64) return fail(XENG_EINVAL, "n_subs %d out of [1, 64]", n_subs);
    for (int k = 0; k < n_subs; ++k) {
        int rc = validate(subs[k], k);
        if (rc) return rc;
    }
    xeng_ctx *ctx = new (std::nothrow) xeng_ctx;
    if (!ctx) return fail(XENG_ENOMEM, "host allocation failed");
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(XENG_EHIP, "hipGetDevice failed");
    }
    ctx->subs.resize(n_subs);
    for (int k = 0; k < n_subs; ++k) {
        Sub &s = ctx->subs[k];
        s.cfg = subs[k];
        s.tri = (int64_t)s.cfg.n_inputs * (s.cfg.n_inputs + 1) / 2;
        s.max_dump = s.cfg.in_bits == 4 ? XENG_MAX_DUMP_SAMPLES_4BIT : XENG_MAX_DUMP_SAMPLES_8BIT;
        s.wt = choose_wt(s.cfg.n_inputs);
        s.bt = 32 * s.wt;
        const int nb = (s.cfg.n_inputs + s.bt - 1) / s.bt;
        s.n_tiles = nb * (nb + 1) / 2;
        const size_t bytes = (size_t)s.tri * (size_t)s.cfg.n_chans * 8;
        hipError_t e = hipMalloc((void **)&s.d_acc, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            xeng_destroy(ctx);
            return fail(XENG_ENOMEM, "hipMalloc(%zu) for subarray %d: %s", bytes, k,
                        hipGetErrorString(e));
        }
        s.acc_zero = true;
    }
    *out = ctx;
    return XENG_OK;
}

int xeng_destroy(xeng_ctx *ctx)
{
    if (!ctx) return XENG_OK;
    int rc = XENG_OK;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(XENG_EHIP, "hipStreamSynchronize failed in destroy");
    for (Sub &s : ctx->subs)
        if (s.d_acc) (void)hipFree(s.d_acc);
    delete ctx;
    return rc;
}

int xeng_set_stream(xeng_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return XENG_OK;
}

int xeng_correlate(xeng_ctx *ctx, const void *const *d_samples)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (!d_samples) return fail(XENG_EINVAL, "d_samples is NULL");
    // all checks first: nothing is launched unless every subarray may proceed
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        const Sub &s = ctx->subs[k];
        if (!d_samples[k]) return fail(XENG_EINVAL, "d_samples[%zu] is NULL", k);
        if (((uintptr_t)d_samples[k] & 3) != 0)
            return fail(XENG_EINVAL, "d_samples[%zu] is not 4-byte aligned", k);
        if (s.since_dump + s.cfg.n_time > s.max_dump)
            return fail(XENG_ERANGE,
                        "subarray %zu: %lld + %d samples since the last dump would exceed the "
                        "exactness bound %lld",
                        k, (long long)s.since_dump, s.cfg.n_time, (long long)s.max_dump);
    }
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        int rc = launch_sub(ctx->subs[k], d_samples[k], ctx->stream);
        if (rc) return rc;
        ctx->subs[k].since_dump += ctx->subs[k].cfg.n_time;
    }
    return XENG_OK;
}

int xeng_dump(xeng_ctx *ctx, void *const *out, int out_is_device, int reset)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (!out && !reset) return fail(XENG_EINVAL, "out is NULL and reset is 0");
    if (out)
        for (size_t k = 0; k < ctx->subs.size(); ++k)
            if (!out[k]) return fail(XENG_EINVAL, "out[%zu] is NULL", k);
    bool host_copy = false;
    for (size_t k = 0; k < ctx->subs.size() && out; ++k) {
        Sub &s = ctx->subs[k];
        const size_t words = (size_t)s.tri * (size_t)s.cfg.n_chans * 2;
        if (s.acc_zero) {
            if (out_is_device) {
                int rc = zero_device((int32_t *)out[k], words, ctx->stream);
                if (rc) return rc;
            } else {
                memset(out[k], 0, words * 4);
            }
        } else {
            HIP_TRY(hipMemcpyAsync(out[k], s.d_acc, words * 4,
                                   out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                   ctx->stream));
            host_copy |= !out_is_device;
        }
    }
    if (host_copy) HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (reset)
        for (Sub &s : ctx->subs) {
            s.acc_zero = true;
            s.since_dump = 0;
        }
    return XENG_OK;
}

int xeng_samples_since_dump(const xeng_ctx *ctx, int sub, int64_t *out)
{
    if (!ctx || !out) return fail(XENG_EINVAL, "NULL argument");
    if (sub < 0 || sub >= (int)ctx->subs.size()) return fail(XENG_EINVAL, "sub %d out of range", sub);
    *out = ctx->subs[sub].since_dump;
    return XENG_OK;
}

int xeng_max_dump_samples(const xeng_ctx *ctx, int sub, int64_t *out)
{
    if (!ctx || !out) return fail(XENG_EINVAL, "NULL argument");
    if (sub < 0 || sub >= (int)ctx->subs.size()) return fail(XENG_EINVAL, "sub %d out of range", sub);
    *out = ctx->subs[sub].max_dump;
    return XENG_OK;
}

int xeng_plan_describe(const xeng_ctx *ctx, char *buf, size_t len)
{
    if (!ctx || !buf) return fail(XENG_EINVAL, "NULL argument");
    std::string js = "{\"subarrays\": [";
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        const Sub &s = ctx->subs[k];
        char item[384];
        const int64_t segs = (s.cfg.n_time + xeng::SEG_T - 1) / xeng::SEG_T;
        snprintf(item, sizeof item,
                 "%s{\"n_inputs\": %d, \"n_chans\": %d, \"n_time\": %d, \"in_bits\": %d, "
                 "\"engine\": \"%s\", \"staging\": \"%s\", \"tile\": %d, \"wave_tile\": %d, \"tiles_per_chan\": %d, "
                 "\"workgroups\": %lld, \"launches_per_call\": %lld}",
                 k ? ", " : "", s.cfg.n_inputs, s.cfg.n_chans, s.cfg.n_time, s.cfg.in_bits,
                 s.cfg.engine == XENG_ENGINE_I8 ? "i8" : "fp8",
                 use_dma(s.cfg.in_bits, s.cfg.n_inputs) ? "lds_dma" : "registers", s.bt, s.bt / 2, s.n_tiles,
                 (long long)s.n_tiles * s.cfg.n_chans, (long long)segs);
        js += item;
    }
    js += "]}";
    if (js.size() + 1 > len) return fail(XENG_EINVAL, "buffer of %zu bytes too small", len);
    memcpy(buf, js.c_str(), js.size() + 1);
    return XENG_OK;
}

} // extern "C"
