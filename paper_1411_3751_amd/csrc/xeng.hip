// libxeng.so: host side of the X-engine C ABI declared in include/xeng.h.
//
// Owns the per-subarray int32 accumulators (packed lower triangle; the
// imaginary words hold Im V_ij - S_i, see xcorr_wg.h, and the dump kernel
// turns them into Im V_ij; a correlate-and-dump writes exact sums straight to
// the caller's output from its last launch), checks the exactness bounds
// before any launch,
// splits each call into segments of at most SEG_T samples, and launches:
//   - 4-bit subarrays with N a multiple of 16 on the int8 engine: the
//     one-wave-per-SIMD kernel (xcorr_w1.h), all such subarrays in one launch
//     over a precomputed, cost-balanced list of half tiles; its accumulator
//     holds the output convention, and a correlate-and-dump writes the
//     caller's output straight from the flush;
//   - other subarrays with N a multiple of 16 (4-bit) or 8 (8-bit): the
//     persistent-workgroup kernel, all such subarrays of one engine and input
//     width in one launch over a precomputed, cost-balanced list of
//     128 x 128 tiles;
//   - other subarrays: the register-staging tile kernel, one launch per
//     subarray and segment.
// The streaming ring (xeng_stream_*) is built on this API in xeng_stream.h.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/xeng.h"
#include "xcorr_i8.h"
#include "xcorr_w1.h"
#include "xcorr_wg.h"
#include "xcorr_sn.h"

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

constexpr int MAX_SUBS = 16;        // subarrays per context (kernel-argument descriptors)
constexpr int WG_PER_CU = 2;        // resident workgroups per CU of the persistent kernel

struct Sub {
    xeng_subarray cfg{};
    int32_t *d_acc = nullptr;  // [F][tri][2], raw convention
    int64_t tri = 0;
    int64_t since_dump = 0;    // samples accumulated since the last reset
    int64_t max_dump = 0;      // exactness bound on since_dump
    bool acc_zero = true;      // accumulator logically zero (next launch overwrites)
    bool wave = false;         // handled by a persistent kernel (one launch per group)
    bool w1 = false;           // ... a wave-private one
    int wv = 0;                // which one: 1 (one wave per SIMD) or 2 (two); 3: the
                               // small-N kernel (one channel per item)
    int wt = 4;                // register kernel: wave tile edge in 16-row sub-blocks
    int bt = 128;              // register kernel: workgroup tile edge
    int n_tiles = 0;           // register kernel: tiles per channel
    int32_t *d_fast = nullptr; // inputs whose autocorrelations have a fast cadence
    int n_fast = 0;
};

// Device memory released by hipFree when its last owner lets go: a plan's
// tile list is owned by its context and by every graph captured with it, so
// replanning (autotuning) never frees memory a graph still launches with.
struct DevFree {
    void operator()(void *p) const
    {
        if (p) (void)hipFree(p);
    }
};
using DevBuf = std::shared_ptr<void>;

// One persistent-kernel launch group: the subarrays it covers and its schedule.
struct WavePlan {
    int engine = XENG_ENGINE_I8;     // every subarray of a plan uses this engine
    int in_bits = 4;                 // and this input width
    bool w1 = false;                 // wave-private kernel (items per wave) or 4-wave kernel (tiles)
    int wv = 0;                      // wave-private kernel: 1 or 2 waves per SIMD; 3: small-N kernel
    std::vector<int> subs;           // context subarray indices, in launch order
    std::vector<xeng::WgItem> items; // flat, grouped per workgroup
    std::vector<int32_t> wg_begin;   // [n_wg + 1]
    int n_wg = 0;
    DevBuf d_mem;                    // one allocation: items, then wg_begin
    xeng::WgItem *d_items = nullptr;
    int32_t *d_wg_begin = nullptr;
    double max_wg_cost = 0, mean_wg_cost = 0;
};

} // namespace

struct xeng_ctx {
    std::vector<Sub> subs;
    std::vector<WavePlan> plans;
    int wg_per_cu = WG_PER_CU;       // persistent launches: workgroups per CU
    int order = 0;                   // persistent schedule: 0 locality, 1 costliest first
    bool tuned = false;              // choices came from the autotuner (or its cache)
    std::string tune_log;            // JSON objects of the last autotune's timings
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 0;
    std::string arch;                // device architecture ("gfx950"): part of the tuning keys
    uint32_t *d_stage = nullptr;  // device staging for host dumps
    size_t stage_words = 0;
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

// Register-staging kernel: whole dword loads when a dword holds whole inputs.
KernelFn pick_kernel(int in_bits, int wt, int n_inputs)
{
    if (in_bits == 4)
        return (n_inputs % 4 == 0) ? pick_wt<4, true>(wt) : pick_wt<4, false>(wt);
    return (n_inputs % 2 == 0) ? pick_wt<8, true>(wt) : pick_wt<8, false>(wt);
}

// Persistent-workgroup kernel: 16-byte copy chunks of whole inputs.
bool wave_path(const xeng_subarray &c)
{
    return (c.in_bits == 4 && c.n_inputs % 16 == 0) || (c.in_bits == 8 && c.n_inputs % 8 == 0);
}

// One-wave kernel: 4-bit input, int8 engine, 16-byte copy chunks of whole inputs.
bool w1_path(const xeng_subarray &c)
{
    return c.in_bits == 4 && c.engine == XENG_ENGINE_I8 && c.n_inputs % 16 == 0;
}

// Small-N kernel: 4-bit input, int8 engine, at most 64 inputs in 16-byte
// chunks, 256-row stages whose byte offsets fit 32 bits.
bool sn_path(const xeng_subarray &c)
{
    return c.in_bits == 4 && c.engine == XENG_ENGINE_I8 && c.n_inputs <= xeng::SN_MAX_N &&
           c.n_inputs % 16 == 0 && (int64_t)c.n_chans * c.n_inputs * xeng::SN_TKS < ((int64_t)1 << 31);
}

int choose_wt(int n_inputs)
{
    if (n_inputs <= 32) return 1;
    if (n_inputs <= 64) return 2;
    return 4;
}

int validate(const xeng_subarray &s, int idx)
{
    if (s.n_inputs < 1 || s.n_inputs > 65535)
        return fail(XENG_EINVAL, "subarray %d: n_inputs %d out of [1, 65535]", idx, s.n_inputs);
    if (s.n_chans < 1 || s.n_chans > (1 << 24) - 1)
        return fail(XENG_EINVAL, "subarray %d: n_chans %d out of [1, 2^24)", idx, s.n_chans);
    if (s.n_time < 1)
        return fail(XENG_EINVAL, "subarray %d: n_time %d < 1", idx, s.n_time);
    if (s.in_bits != 4 && s.in_bits != 8)
        return fail(XENG_EINVAL, "subarray %d: in_bits %d is not 4 or 8", idx, s.in_bits);
    if (s.engine != XENG_ENGINE_I8 && s.engine != XENG_ENGINE_FP8)
        return fail(XENG_EINVAL, "subarray %d: unknown engine %d", idx, s.engine);
    if (s.engine == XENG_ENGINE_FP8 && s.in_bits != 4)
        return fail(XENG_EINVAL, "subarray %d: the FP8 engine takes 4-bit input only", idx);
    if (s.engine == XENG_ENGINE_FP8 && s.n_inputs % 16 != 0)
        return fail(XENG_EINVAL, "subarray %d: the FP8 engine needs n_inputs a multiple of 16 (got %d)",
                    idx, s.n_inputs);
    const int64_t tri = (int64_t)s.n_inputs * (s.n_inputs + 1) / 2;
    if (tri * (int64_t)s.n_chans * 2 > ((int64_t)1 << 40))
        return fail(XENG_EINVAL, "subarray %d: output too large", idx);
    // one stage spans TK time rows of the whole [F][N] plane; its byte
    // offsets must fit the 32-bit buffer offsets
    if ((int64_t)s.n_chans * s.n_inputs * (s.in_bits / 4) * xeng::TK >= ((int64_t)1 << 31))
        return fail(XENG_EINVAL, "subarray %d: n_chans * n_inputs too large for one stream", idx);
    const int64_t bound = s.in_bits == 4 ? XENG_MAX_DUMP_SAMPLES_4BIT : XENG_MAX_DUMP_SAMPLES_8BIT;
    if (s.n_time > bound)
        return fail(XENG_EINVAL, "subarray %d: n_time %d above the dump limit %lld", idx, s.n_time,
                    (long long)bound);
    return XENG_OK;
}

// ---- schedule of the persistent-workgroup kernel ------------------------
//
// Tiles (subarray, channel, 128-input block I, block J <= I) are listed in
// locality order (subarray, channel, I, J). The list is cut into 8
// contiguous parts of equal cost, one per XCD (workgroup b runs on XCD
// b mod 8). Within an XCD the tiles are dealt out in rounds of one tile per
// workgroup, so that the workgroups of an XCD work on neighbouring tiles (the
// same channels, at the same times, whose rows they share in that XCD's L2);
// inside a round the costliest tile goes to the least-loaded workgroup.
void build_schedule(WavePlan &p, const std::vector<Sub> &subs, int n_cu, int wg_per_cu, int order)
{
    struct It {
        xeng::WgItem w;
        double cost;
    };
    std::vector<It> all;
    for (size_t k = 0; k < p.subs.size() && p.w1; ++k) {
        // wave-private kernels. One wave per SIMD: tiles of 128, an
        // off-diagonal tile as two J halves (8 MFMA blocks per K step), a
        // diagonal tile as two parts of 5 blocks. Two waves per SIMD: tiles
        // of 64, one item each (4 blocks, or 3 on the diagonal).
        const Sub &s = subs[p.subs[k]];
        const int tile = p.wv == 1 ? 128 : 64;
        const int parts = p.wv == 1 ? 2 : 1;
        const int nb = (s.cfg.n_inputs + tile - 1) / tile;
        const int nst = (s.cfg.n_time + xeng::W1_TK - 1) / xeng::W1_TK;
        const int segs = (s.cfg.n_time + xeng::SEG_T - 1) / xeng::SEG_T;
        const double per_seg = (double)nst / segs;
        for (int f = 0; f < s.cfg.n_chans; ++f)
            for (int bi = 0; bi < nb; ++bi)
                for (int bj = 0; bj <= bi; ++bj)
                    for (int r = 0; r < parts; ++r) {
                        It it;
                        it.w.cs = (uint32_t)f | ((uint32_t)k << 24);
                        const uint32_t role = bi == bj ? 2u + (uint32_t)r : (uint32_t)r;
                        it.w.ij = (uint32_t)bi | ((uint32_t)bj << 12) | (role << 24);
                        // K steps times MFMA blocks, plus the flush
                        const double blocks = p.wv == 1 ? (bi == bj ? 5.0 : 8.0) : (bi == bj ? 3.0 : 4.0);
                        it.cost = per_seg * blocks + 3.0 * blocks;
                        all.push_back(it);
                    }
    }
    for (size_t k = 0; k < p.subs.size() && p.wv == 3; ++k) {
        // small-N kernel: one item per channel, one stage loop per 256 samples
        const Sub &s = subs[p.subs[k]];
        const int nst = (s.cfg.n_time + xeng::SN_TKS - 1) / xeng::SN_TKS;
        const int segs = (s.cfg.n_time + xeng::SEG_T - 1) / xeng::SEG_T;
        for (int f = 0; f < s.cfg.n_chans; ++f) {
            It it;
            it.w.cs = (uint32_t)f | ((uint32_t)k << 24);
            it.w.ij = 0;
            it.cost = (double)nst / segs + 4.0;
            all.push_back(it);
        }
    }
    for (size_t k = 0; k < p.subs.size() && !p.w1 && p.wv != 3; ++k) {
        const Sub &s = subs[p.subs[k]];
        const int nb = (s.cfg.n_inputs + 127) / 128;
        const int tks = s.cfg.in_bits == 4 ? xeng::WgGeom<4>::TKS : xeng::WgGeom<8>::TKS;
        const int nst = (s.cfg.n_time + tks - 1) / tks;
        const int segs = (s.cfg.n_time + xeng::SEG_T - 1) / xeng::SEG_T;
        const double per_stage = (double)nst / segs;
        for (int f = 0; f < s.cfg.n_chans; ++f)
            for (int bi = 0; bi < nb; ++bi)
                for (int bj = 0; bj <= bi; ++bj) {
                    It it;
                    it.w.cs = (uint32_t)f | ((uint32_t)k << 24);
                    it.w.ij = (uint32_t)bi | ((uint32_t)bj << 16);
                    // a stage loop per stage (the busiest wave of a diagonal
                    // tile has 2.5 or 3 MFMA tiles, off the diagonal 4, and
                    // the loop's other work is the same; 0.66 timed the same
                    // as 0.75 with 2.5), plus a per-tile flush
                    it.cost = per_stage * (bi == bj ? 0.75 : 1.0) + 2.0;
                    all.push_back(it);
                }
    }
    // order 1: costliest tiles first (the list is still cut into contiguous
    // per-XCD parts, which then hold similar-cost tiles)
    if (order == 1)
        std::stable_sort(all.begin(), all.end(), [](const It &a, const It &b) { return a.cost > b.cost; });
    const int64_t n_items = (int64_t)all.size();
    const int per_cu = p.w1 ? (p.wv == 1 ? xeng::W1Geo<1>::WG_PER_CU : xeng::W1Geo<2>::WG_PER_CU)
                            : wg_per_cu;
    const int n_wg = (int)std::min<int64_t>((int64_t)n_cu * per_cu, n_items);
    p.n_wg = n_wg;
    std::vector<std::vector<int>> xwg(8);
    for (int b = 0; b < n_wg; ++b) xwg[b % 8].push_back(b);
    const double total = std::accumulate(all.begin(), all.end(), 0.0,
                                         [](double acc, const It &i) { return acc + i.cost; });
    std::vector<std::vector<xeng::WgItem>> per_wg(n_wg);
    std::vector<double> load(n_wg, 0.0);
    int64_t pos = 0;
    double cum = 0.0, cum_target = 0.0;
    for (int x = 0; x < 8; ++x) {
        if (xwg[x].empty()) continue;
        cum_target += total * (double)xwg[x].size() / (double)n_wg;
        const int64_t first = pos;
        while (pos < n_items && (x == 7 || cum + all[pos].cost * 0.5 <= cum_target)) {
            cum += all[pos].cost;
            ++pos;
        }
        const std::vector<int> &ws = xwg[x];
        for (int64_t r0 = first; r0 < pos; r0 += (int64_t)ws.size()) {
            const int64_t r1 = std::min<int64_t>(pos, r0 + (int64_t)ws.size());
            std::vector<int64_t> idx(r1 - r0);
            std::iota(idx.begin(), idx.end(), r0);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int64_t a, int64_t b) { return all[a].cost > all[b].cost; });
            std::vector<int> wv(ws);
            std::stable_sort(wv.begin(), wv.end(), [&](int a, int b) { return load[a] < load[b]; });
            for (size_t q = 0; q < idx.size(); ++q) {
                per_wg[wv[q]].push_back(all[idx[q]].w);
                load[wv[q]] += all[idx[q]].cost;
            }
        }
    }
    p.items.clear();
    p.wg_begin.assign(1, 0);
    for (int b = 0; b < n_wg; ++b) {
        p.items.insert(p.items.end(), per_wg[b].begin(), per_wg[b].end());
        p.wg_begin.push_back((int32_t)p.items.size());
    }
    p.max_wg_cost = *std::max_element(load.begin(), load.end());
    p.mean_wg_cost = total / n_wg;
}

int upload_plan(WavePlan &p)
{
    const size_t item_bytes = (sizeof(xeng::WgItem) * std::max<size_t>(1, p.items.size()) + 255) & ~(size_t)255;
    const size_t total = item_bytes + sizeof(int32_t) * p.wg_begin.size();
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XENG_ENOMEM, "hipMalloc(%zu) for a tile list: %s", total, hipGetErrorString(e));
    }
    p.d_mem = DevBuf(mem, DevFree());
    p.d_items = (xeng::WgItem *)mem;
    p.d_wg_begin = (int32_t *)((char *)mem + item_bytes);
    HIP_TRY(hipMemcpy(p.d_items, p.items.data(), sizeof(xeng::WgItem) * p.items.size(),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p.d_wg_begin, p.wg_begin.data(), sizeof(int32_t) * p.wg_begin.size(),
                      hipMemcpyHostToDevice));
    return XENG_OK;
}

int zero_device(uint32_t *p, size_t n_words, hipStream_t st)
{
    const size_t n16 = n_words / 4, ntail = n_words % 4;
    int blocks = (int)((n16 + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(xeng::fill_zero_kernel, dim3(blocks), dim3(256), 0, st, (int4 *)p, n16,
                       (int32_t *)p + n16 * 4, ntail);
    HIP_TRY(hipGetLastError());
    return XENG_OK;
}

int launch_regs(Sub &s, const void *d_samples, hipStream_t st)
{
    const xeng_subarray &c = s.cfg;
    KernelFn fn = pick_kernel(c.in_bits, s.wt, c.n_inputs);
    for (int64_t t0 = 0; t0 < c.n_time; t0 += xeng::SEG_T) {
        xeng::TileArgs a;
        a.samples = (const uint8_t *)d_samples;
        a.vis = s.d_acc;
        a.t_begin = t0;
        a.t_count = (int32_t)std::min<int64_t>(c.n_time - t0, xeng::SEG_T);
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

// One-wave kernel. out == NULL: every segment integrates into the
// accumulators. out != NULL (a correlate-and-dump with reset): the last
// segment's flush writes subarray k's sums to out[k] instead, and the
// accumulator is left as it was (the caller resets it).
int launch_w1(xeng_ctx *ctx, WavePlan &p, const void *const *d_samples, void *const *out)
{
    const Sub &s0 = ctx->subs[p.subs[0]];
    const int64_t T = s0.cfg.n_time;
    for (int64_t t0 = 0; t0 < T; t0 += xeng::SEG_T) {
        const bool last = t0 + xeng::SEG_T >= T;
        xeng::W1Args a;
        memset(&a, 0, sizeof a);
        for (size_t k = 0; k < p.subs.size(); ++k) {
            Sub &s = ctx->subs[p.subs[k]];
            xeng::W1Sub &w = a.subs[k];
            w.samples = (const uint8_t *)d_samples[p.subs[k]];
            w.src = s.acc_zero ? nullptr : s.d_acc;
            w.dst = (last && out) ? (int32_t *)out[p.subs[k]] : s.d_acc;
            w.t_begin = t0;
            w.t_count = (int32_t)std::min<int64_t>(s.cfg.n_time - t0, xeng::SEG_T);
            w.n_chans = s.cfg.n_chans;
            w.n_inputs = s.cfg.n_inputs;
        }
        a.items = p.d_items;
        a.wg_begin = p.d_wg_begin;
        if (p.wv == 1)
            hipLaunchKernelGGL(xeng::xcorr_w1_kernel<1>, dim3(p.n_wg), dim3(64), 0, ctx->stream, a);
        else
            hipLaunchKernelGGL(xeng::xcorr_w1_kernel<2>, dim3(p.n_wg), dim3(64), 0, ctx->stream, a);
        HIP_TRY(hipGetLastError());
        if (!(last && out))
            for (int k : p.subs) ctx->subs[k].acc_zero = false;
    }
    return XENG_OK;
}

// Persistent kernels (all subarrays of a plan have the same number of
// segments: a plan with several subarrays is only built when every one fits
// in one segment). out == NULL: every segment integrates into the
// accumulators. out != NULL (a correlate-and-dump with reset): the last
// segment's flush writes subarray k's sums to out[k] instead, and the
// accumulator is left as it was (the caller resets it).
int launch_wave(xeng_ctx *ctx, WavePlan &p, const void *const *d_samples, void *const *out = nullptr)
{
    if (p.w1) return launch_w1(ctx, p, d_samples, out);
    const Sub &s0 = ctx->subs[p.subs[0]];
    const int64_t T = s0.cfg.n_time;
    for (int64_t t0 = 0; t0 < T; t0 += xeng::SEG_T) {
        const bool last = t0 + xeng::SEG_T >= T;
        xeng::WgArgs a;
        memset(&a, 0, sizeof a);
        for (size_t k = 0; k < p.subs.size(); ++k) {
            Sub &s = ctx->subs[p.subs[k]];
            xeng::WgSub &w = a.subs[k];
            w.samples = (const uint8_t *)d_samples[p.subs[k]];
            w.src = s.acc_zero ? nullptr : s.d_acc;
            w.dst = (last && out) ? (int32_t *)out[p.subs[k]] : s.d_acc;
            w.t_begin = t0;
            w.t_count = (int32_t)std::min<int64_t>(s.cfg.n_time - t0, xeng::SEG_T);
            w.n_chans = s.cfg.n_chans;
            w.n_inputs = s.cfg.n_inputs;
        }
        a.items = p.d_items;
        a.wg_begin = p.d_wg_begin;
        // the launch that writes the caller's output sums S_i and writes exact
        // sums; the others leave the raw form in the accumulator
        const bool fuse = last && out;
        const dim3 g(p.n_wg), b(xeng::WG_THREADS);
        if (p.wv == 3) {
            if (fuse) hipLaunchKernelGGL((xeng::xcorr_sn_kernel<true>), g, b, 0, ctx->stream, a);
            else hipLaunchKernelGGL((xeng::xcorr_sn_kernel<false>), g, b, 0, ctx->stream, a);
        } else if (p.engine == XENG_ENGINE_FP8) {
            if (fuse) hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_F8, 4, true>), g, b, 0, ctx->stream, a);
            else hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_F8, 4, false>), g, b, 0, ctx->stream, a);
        } else if (p.in_bits == 4) {
            if (fuse) hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 4, true>), g, b, 0, ctx->stream, a);
            else hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 4, false>), g, b, 0, ctx->stream, a);
        } else {
            if (fuse) hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 8, true>), g, b, 0, ctx->stream, a);
            else hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 8, false>), g, b, 0, ctx->stream, a);
        }
        HIP_TRY(hipGetLastError());
        if (!(last && out))
            for (int k : p.subs) ctx->subs[k].acc_zero = false;
    }
    return XENG_OK;
}

// Every accumulator is in the raw form (exact sums are raw sums with a zero
// diagonal), so one dump kernel serves all kernel families.
int dump_device(const Sub &s, uint32_t *out, hipStream_t st)
{
    const unsigned gx = (unsigned)((s.tri + xeng::DUMP_PER_WG - 1) / xeng::DUMP_PER_WG);
    for (int c0 = 0; c0 < s.cfg.n_chans; c0 += 65535) {
        const int nc = std::min(65535, s.cfg.n_chans - c0);
        hipLaunchKernelGGL(xeng::dump_kernel, dim3(gx, (unsigned)nc), dim3(256), 0, st,
                           (const uint2 *)s.d_acc, (uint2 *)out, (int32_t)s.tri, c0);
        HIP_TRY(hipGetLastError());
    }
    return XENG_OK;
}

// Drops the context's hold on its tile lists (a graph may still hold them).
void free_plans(xeng_ctx *ctx) { ctx->plans.clear(); }

// Launch groups of the persistent kernel from the subarrays' kernel choices:
// per (engine, input width), one group for all its subarrays when each fits
// one segment, otherwise one group per subarray.
int replan(xeng_ctx *ctx)
{
    free_plans(ctx);
    for (Sub &s : ctx->subs) {
        const int nb = (s.cfg.n_inputs + s.bt - 1) / s.bt;
        s.n_tiles = nb * (nb + 1) / 2;
    }
    // (engine, input width, wave-private kernel variant)
    const int kinds[6][3] = {{XENG_ENGINE_I8, 4, 3}, {XENG_ENGINE_I8, 4, 1}, {XENG_ENGINE_I8, 4, 2},
                             {XENG_ENGINE_I8, 4, 0}, {XENG_ENGINE_I8, 8, 0}, {XENG_ENGINE_FP8, 4, 0}};
    for (const auto &kd : kinds) {
        std::vector<int> es;
        bool one_group = true;
        for (int k = 0; k < (int)ctx->subs.size(); ++k) {
            const Sub &s = ctx->subs[k];
            if (s.wave && s.cfg.engine == kd[0] && s.cfg.in_bits == kd[1] && s.wv == kd[2]) {
                es.push_back(k);
                if (s.cfg.n_time > xeng::SEG_T) one_group = false;
            }
        }
        if (es.empty()) continue;
        std::vector<std::vector<int>> groups;
        if (one_group) groups.push_back(es);
        else
            for (int k : es) groups.push_back({k});
        for (auto &g : groups) {
            ctx->plans.emplace_back();
            ctx->plans.back().engine = kd[0];
            ctx->plans.back().in_bits = kd[1];
            ctx->plans.back().w1 = kd[2] == 1 || kd[2] == 2;
            ctx->plans.back().wv = kd[2];
            ctx->plans.back().subs = g;
        }
    }
    for (WavePlan &p : ctx->plans) {
        build_schedule(p, ctx->subs, ctx->n_cu, ctx->wg_per_cu, ctx->order);
        int rc = upload_plan(p);
        if (rc) return rc;
    }
    return XENG_OK;
}

// ---- tuning cache: choices found by xeng_autotune, per subarray shape and
// per set of shapes (the schedule of a batched launch), for this process.
struct SubKey {
    int n, f, t, b, e;
    bool operator<(const SubKey &o) const
    {
        return std::tie(n, f, t, b, e) < std::tie(o.n, o.f, o.t, o.b, o.e);
    }
};
// Kernel families: register-staging tiles, the persistent 4-wave kernel, the
// wave-private kernel with one or two waves per SIMD, the small-N kernel.
constexpr int FAM_REG = 0, FAM_WG = 1, FAM_W1 = 2, FAM_W2 = 3, FAM_SN = 4;
struct SubChoice {
    int fam;
    int wt;
};
struct SchedChoice {
    int wg_per_cu, order;
};
// Keys carry the device architecture: choices measured on one chip are not
// applied on another.
using ArchKey = std::pair<std::string, SubKey>;
using ArchSet = std::pair<std::string, std::vector<SubKey>>;
std::mutex g_tune_mu;
std::map<ArchKey, SubChoice> g_tune_sub;
std::map<ArchSet, SchedChoice> g_tune_sched;
// per set of shapes: the choices of a batch tuned as a whole
std::map<ArchSet, std::vector<SubChoice>> g_tune_set;

SubKey key_of(const xeng_subarray &c) { return SubKey{c.n_inputs, c.n_chans, c.n_time, c.in_bits, c.engine}; }

std::vector<SubKey> keys_of(const xeng_ctx *ctx)
{
    std::vector<SubKey> v;
    for (const Sub &s : ctx->subs) v.push_back(key_of(s.cfg));
    return v;
}

// The best family a subarray can take: fam, or the next one down that
// supports its shape and engine (the FP8 engine exists only in the 4-wave
// kernel).
void set_choice(Sub &s, int fam, int wt)
{
    if (s.cfg.engine == XENG_ENGINE_FP8) fam = FAM_WG;
    if ((fam == FAM_W1 || fam == FAM_W2) && !w1_path(s.cfg)) fam = FAM_WG;
    if (fam == FAM_SN && !sn_path(s.cfg)) fam = FAM_WG;
    if (fam == FAM_WG && !wave_path(s.cfg)) fam = FAM_REG;
    s.wave = fam != FAM_REG;
    s.w1 = fam == FAM_W1 || fam == FAM_W2;
    s.wv = fam == FAM_W1 ? 1 : (fam == FAM_W2 ? 2 : (fam == FAM_SN ? 3 : 0));
    s.wt = wt;
    s.bt = 32 * wt;
    // the register-staging launch's grid follows the tile size
    const int nb = (s.cfg.n_inputs + s.bt - 1) / s.bt;
    s.n_tiles = nb * (nb + 1) / 2;
}

const char *fam_name(int fam)
{
    return fam == FAM_W1   ? "one_wave"
           : fam == FAM_W2 ? "two_wave"
           : fam == FAM_SN ? "small_n"
           : fam == FAM_WG ? "persistent_workgroup"
                           : "register_staging";
}

int fam_of(const Sub &s)
{
    return s.wv == 1 ? FAM_W1 : (s.wv == 2 ? FAM_W2 : (s.wv == 3 ? FAM_SN : (s.wave ? FAM_WG : FAM_REG)));
}

void apply_tuning_cache(xeng_ctx *ctx)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool all = true;
    auto set_it = g_tune_set.find(ArchSet{ctx->arch, keys_of(ctx)});
    if (set_it != g_tune_set.end()) {
        for (size_t k = 0; k < ctx->subs.size(); ++k)
            set_choice(ctx->subs[k], set_it->second[k].fam, set_it->second[k].wt);
    } else {
        for (Sub &s : ctx->subs) {
            auto it = g_tune_sub.find(ArchKey{ctx->arch, key_of(s.cfg)});
            if (it == g_tune_sub.end()) {
                all = false;
                continue;
            }
            set_choice(s, it->second.fam, it->second.wt);
        }
    }
    auto it = g_tune_sched.find(ArchSet{ctx->arch, keys_of(ctx)});
    if (it != g_tune_sched.end()) {
        ctx->wg_per_cu = it->second.wg_per_cu;
        ctx->order = it->second.order;
    }
    ctx->tuned = all && it != g_tune_sched.end();
}

void free_ctx(xeng_ctx *ctx)
{
    for (Sub &s : ctx->subs) {
        if (s.d_acc) (void)hipFree(s.d_acc);
        if (s.d_fast) (void)hipFree(s.d_fast);
    }
    free_plans(ctx);
    if (ctx->d_stage) (void)hipFree(ctx->d_stage);
    delete ctx;
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
    case XENG_EBUSY: return "no free ring slot (gulp dropped)";
    default: return "unknown error";
    }
}

const char *xeng_last_error(void) { return g_last_error.c_str(); }

int xeng_set_fast_autos(xeng_ctx *ctx, int sub, const int32_t *inputs, int n)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (sub < 0 || sub >= (int)ctx->subs.size()) return fail(XENG_EINVAL, "sub %d out of range", sub);
    if (n < 0 || (n > 0 && !inputs)) return fail(XENG_EINVAL, "bad input list");
    Sub &s = ctx->subs[sub];
    if (n > s.cfg.n_inputs) return fail(XENG_EINVAL, "%d inputs selected of %d", n, s.cfg.n_inputs);
    for (int q = 0; q < n; ++q)
        if (inputs[q] < 0 || inputs[q] >= s.cfg.n_inputs)
            return fail(XENG_EINVAL, "input %d out of [0, %d)", inputs[q], s.cfg.n_inputs);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (s.d_fast) (void)hipFree(s.d_fast);
    s.d_fast = nullptr;
    s.n_fast = 0;
    if (n == 0) return XENG_OK;
    hipError_t e = hipMalloc((void **)&s.d_fast, sizeof(int32_t) * (size_t)n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XENG_ENOMEM, "hipMalloc for the fast-cadence input list: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpy(s.d_fast, inputs, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
    s.n_fast = n;
    return XENG_OK;
}

int xeng_dump_fast_autos(xeng_ctx *ctx, void *const *out, int out_is_device, int reset)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (!out && !reset) return fail(XENG_EINVAL, "out is NULL and reset is 0");
    if (out && !out_is_device) return fail(XENG_EINVAL, "fast-cadence dumps go to device memory");
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        Sub &s = ctx->subs[k];
        if (s.n_fast == 0) continue;
        if (out && !out[k]) return fail(XENG_EINVAL, "out[%zu] is NULL", k);
        const int64_t total = (int64_t)s.cfg.n_chans * s.n_fast;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(xeng::fast_autos_kernel, dim3(blocks), dim3(256), 0, ctx->stream,
                           (uint2 *)s.d_acc, s.tri, s.cfg.n_chans, s.d_fast, s.n_fast,
                           out ? (int32_t *)out[k] : (int32_t *)nullptr, reset ? 1 : 0,
                           s.acc_zero ? 1 : 0);
        HIP_TRY(hipGetLastError());
    }
    return XENG_OK;
}

} // extern "C"
namespace {
std::string device_arch(int dev);
void tuning_file_autoload();
void tuning_file_autosave();
} // namespace
extern "C" {

int xeng_create(const xeng_subarray *subs, int n_subs, void *hip_stream, xeng_ctx **out)
{
    if (!out) return fail(XENG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!subs) return fail(XENG_EINVAL, "subs is NULL");
    if (n_subs < 1 || n_subs > MAX_SUBS)
        return fail(XENG_EINVAL, "n_subs %d out of [1, %d]", n_subs, MAX_SUBS);
    for (int k = 0; k < n_subs; ++k) {
        int rc = validate(subs[k], k);
        if (rc) return rc;
    }
    xeng_ctx *ctx = new (std::nothrow) xeng_ctx;
    if (!ctx) return fail(XENG_ENOMEM, "host allocation failed");
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
            hipSuccess ||
        ctx->n_cu < 1) {
        delete ctx;
        return fail(XENG_EHIP, "cannot query the current HIP device");
    }
    ctx->arch = device_arch(ctx->device);
    tuning_file_autoload();
    ctx->subs.resize(n_subs);
    for (int k = 0; k < n_subs; ++k) {
        Sub &s = ctx->subs[k];
        s.cfg = subs[k];
        s.tri = (int64_t)s.cfg.n_inputs * (s.cfg.n_inputs + 1) / 2;
        s.max_dump = s.cfg.in_bits == 4 ? XENG_MAX_DUMP_SAMPLES_4BIT : XENG_MAX_DUMP_SAMPLES_8BIT;
        set_choice(s, sn_path(s.cfg) ? FAM_SN : FAM_WG, choose_wt(s.cfg.n_inputs));
        const int nb = (s.cfg.n_inputs + s.bt - 1) / s.bt;
        s.n_tiles = nb * (nb + 1) / 2;
        const size_t bytes = (size_t)s.tri * (size_t)s.cfg.n_chans * 8;
        hipError_t e = hipMalloc((void **)&s.d_acc, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_ctx(ctx);
            return fail(XENG_ENOMEM, "hipMalloc(%zu) for subarray %d: %s", bytes, k,
                        hipGetErrorString(e));
        }
    }
    apply_tuning_cache(ctx);
    int rc = replan(ctx);
    if (rc) {
        free_ctx(ctx);
        return rc;
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
    free_ctx(ctx);
    return rc;
}

int xeng_set_stream(xeng_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    hipStream_t next = (hipStream_t)hip_stream;
    if (next != ctx->stream) {
        // work already queued on the old stream comes first on the new one
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ev, ctx->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess)
            return fail(XENG_EHIP, "ordering the new stream after the old: %s", hipGetErrorString(e));
    }
    ctx->stream = next;
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
        if (((uintptr_t)d_samples[k] & 15) != 0)
            return fail(XENG_EINVAL, "d_samples[%zu] is not 16-byte aligned", k);
        if (s.since_dump + s.cfg.n_time > s.max_dump)
            return fail(XENG_ERANGE,
                        "subarray %zu: %lld + %d samples since the last dump would exceed the "
                        "exactness bound %lld",
                        k, (long long)s.since_dump, s.cfg.n_time, (long long)s.max_dump);
    }
    for (WavePlan &p : ctx->plans) {
        int rc = launch_wave(ctx, p, d_samples);
        if (rc) return rc;
    }
    for (size_t k = 0; k < ctx->subs.size(); ++k)
        if (!ctx->subs[k].wave) {
            int rc = launch_regs(ctx->subs[k], d_samples[k], ctx->stream);
            if (rc) return rc;
        }
    for (Sub &s : ctx->subs) s.since_dump += s.cfg.n_time;
    return XENG_OK;
}

int xeng_dump(xeng_ctx *ctx, void *const *out, int out_is_device, int reset)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (!out && !reset) return fail(XENG_EINVAL, "out is NULL and reset is 0");
    if (out)
        for (size_t k = 0; k < ctx->subs.size(); ++k)
            if (!out[k]) return fail(XENG_EINVAL, "out[%zu] is NULL", k);
    for (size_t k = 0; k < ctx->subs.size() && out; ++k) {
        Sub &s = ctx->subs[k];
        const size_t words = (size_t)s.tri * (size_t)s.cfg.n_chans * 2;
        if (s.acc_zero) {
            if (out_is_device) {
                int rc = zero_device((uint32_t *)out[k], words, ctx->stream);
                if (rc) return rc;
            } else {
                HIP_TRY(hipStreamSynchronize(ctx->stream));
                memset(out[k], 0, words * 4);
            }
        } else if (out_is_device) {
            int rc = dump_device(s, (uint32_t *)out[k], ctx->stream);
            if (rc) return rc;
        } else {
            if (ctx->stage_words < words) {
                HIP_TRY(hipStreamSynchronize(ctx->stream));
                if (ctx->d_stage) (void)hipFree(ctx->d_stage);
                ctx->d_stage = nullptr;
                ctx->stage_words = 0;
                hipError_t e = hipMalloc((void **)&ctx->d_stage, words * 4);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(XENG_ENOMEM, "hipMalloc(%zu) for the dump staging buffer: %s",
                                words * 4, hipGetErrorString(e));
                }
                ctx->stage_words = words;
            }
            int rc = dump_device(s, ctx->d_stage, ctx->stream);
            if (rc) return rc;
            HIP_TRY(hipMemcpyAsync(out[k], ctx->d_stage, words * 4, hipMemcpyDeviceToHost,
                                   ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
        }
    }
    if (reset)
        for (Sub &s : ctx->subs) {
            s.acc_zero = true;
            s.since_dump = 0;
        }
    return XENG_OK;
}

int xeng_correlate_dump(xeng_ctx *ctx, const void *const *d_samples, void *const *out,
                        int out_is_device, int reset)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (!(out && out_is_device && reset)) {
        // nothing to fuse: the two calls in order
        int rc = xeng_correlate(ctx, d_samples);
        if (rc) return rc;
        return xeng_dump(ctx, out, out_is_device, reset);
    }
    if (!d_samples) return fail(XENG_EINVAL, "d_samples is NULL");
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        const Sub &s = ctx->subs[k];
        if (!d_samples[k]) return fail(XENG_EINVAL, "d_samples[%zu] is NULL", k);
        if (((uintptr_t)d_samples[k] & 15) != 0)
            return fail(XENG_EINVAL, "d_samples[%zu] is not 16-byte aligned", k);
        if (!out[k]) return fail(XENG_EINVAL, "out[%zu] is NULL", k);
        if (s.since_dump + s.cfg.n_time > s.max_dump)
            return fail(XENG_ERANGE,
                        "subarray %zu: %lld + %d samples since the last dump would exceed the "
                        "exactness bound %lld",
                        k, (long long)s.since_dump, s.cfg.n_time, (long long)s.max_dump);
    }
    // the persistent kernels write their last segment straight to out; the
    // register-staging kernel integrates and is dumped
    for (WavePlan &p : ctx->plans) {
        int rc = launch_wave(ctx, p, d_samples, out);
        if (rc) return rc;
    }
    for (size_t k = 0; k < ctx->subs.size(); ++k)
        if (!ctx->subs[k].wave) {
            int rc = launch_regs(ctx->subs[k], d_samples[k], ctx->stream);
            if (rc) return rc;
        }
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        Sub &s = ctx->subs[k];
        if (s.wave) continue;
        int rc = dump_device(s, (uint32_t *)out[k], ctx->stream);
        if (rc) return rc;
    }
    for (Sub &s : ctx->subs) {
        s.acc_zero = true;
        s.since_dump = 0;
    }
    return XENG_OK;
}

int xeng_set_kernel(xeng_ctx *ctx, int sub, int kernel, int tile)
{
    if (!ctx) return fail(XENG_EINVAL, "ctx is NULL");
    if (sub < 0 || sub >= (int)ctx->subs.size()) return fail(XENG_EINVAL, "sub %d out of range", sub);
    if (kernel < XENG_KERNEL_REGISTER || kernel > XENG_KERNEL_SMALL_N)
        return fail(XENG_EINVAL, "unknown kernel family %d", kernel);
    if (kernel == XENG_KERNEL_REGISTER && tile != 32 && tile != 64 && tile != 128)
        return fail(XENG_EINVAL, "register-staging tile %d is not 32, 64 or 128", tile);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const int fam = kernel == XENG_KERNEL_REGISTER ? FAM_REG
                    : kernel == XENG_KERNEL_PERSISTENT ? FAM_WG
                    : kernel == XENG_KERNEL_ONE_WAVE ? FAM_W1
                    : kernel == XENG_KERNEL_TWO_WAVE ? FAM_W2 : FAM_SN;
    Sub &s = ctx->subs[sub];
    set_choice(s, fam, kernel == XENG_KERNEL_REGISTER ? tile / 32 : s.wt);
    int rc = replan(ctx);
    if (rc) return rc;
    for (Sub &t : ctx->subs) {
        t.acc_zero = true;
        t.since_dump = 0;
    }
    ctx->tuned = false;
    return XENG_OK;
}

int xeng_samples_since_dump(const xeng_ctx *ctx, int sub, int64_t *out)
{
    if (!ctx || !out) return fail(XENG_EINVAL, "NULL argument");
    if (sub < 0 || sub >= (int)ctx->subs.size())
        return fail(XENG_EINVAL, "sub %d out of range", sub);
    *out = ctx->subs[sub].since_dump;
    return XENG_OK;
}

int xeng_max_dump_samples(const xeng_ctx *ctx, int sub, int64_t *out)
{
    if (!ctx || !out) return fail(XENG_EINVAL, "NULL argument");
    if (sub < 0 || sub >= (int)ctx->subs.size())
        return fail(XENG_EINVAL, "sub %d out of range", sub);
    *out = ctx->subs[sub].max_dump;
    return XENG_OK;
}

int xeng_plan_describe(const xeng_ctx *ctx, char *buf, size_t len)
{
    if (!ctx || !buf) return fail(XENG_EINVAL, "NULL argument");
    std::string js = "{\"compute_units\": " + std::to_string(ctx->n_cu) + ", \"subarrays\": [";
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        const Sub &s = ctx->subs[k];
        char item[512];
        const int64_t segs = (s.cfg.n_time + xeng::SEG_T - 1) / xeng::SEG_T;
        if (s.wave)
            snprintf(item, sizeof item,
                     "%s{\"n_inputs\": %d, \"n_chans\": %d, \"n_time\": %d, \"in_bits\": %d, "
                     "\"engine\": \"%s\", \"kernel\": \"%s\", \"tile\": %d, "
                     "\"launches_per_call\": %lld}",
                     k ? ", " : "", s.cfg.n_inputs, s.cfg.n_chans, s.cfg.n_time, s.cfg.in_bits,
                     s.cfg.engine == XENG_ENGINE_I8 ? "i8" : "fp8", fam_name(fam_of(s)),
                     s.wv == 2 || s.wv == 3 ? 64 : 128, (long long)segs);
        else
            snprintf(item, sizeof item,
                     "%s{\"n_inputs\": %d, \"n_chans\": %d, \"n_time\": %d, \"in_bits\": %d, "
                     "\"engine\": \"%s\", \"kernel\": \"register_staging\", \"tile\": %d, "
                     "\"wave_tile\": %d, \"tiles_per_chan\": %d, \"workgroups\": %lld, "
                     "\"launches_per_call\": %lld}",
                     k ? ", " : "", s.cfg.n_inputs, s.cfg.n_chans, s.cfg.n_time, s.cfg.in_bits,
                     s.cfg.engine == XENG_ENGINE_I8 ? "i8" : "fp8", s.bt, s.bt / 2, s.n_tiles,
                     (long long)s.n_tiles * s.cfg.n_chans, (long long)segs);
        js += item;
    }
    js += "], \"tuned\": " + std::string(ctx->tuned ? "true" : "false") +
          ", \"workgroups_per_cu\": " + std::to_string(ctx->wg_per_cu) +
          ", \"schedule_order\": \"" + (ctx->order ? "costliest_first" : "locality") + "\"";
    js += ", \"persistent_launch_groups\": [";
    for (size_t q = 0; q < ctx->plans.size(); ++q) {
        const WavePlan &p = ctx->plans[q];
        char item[256];
        snprintf(item, sizeof item,
                 "%s{\"kernel\": \"%s\", \"subarrays\": %zu, \"items\": %zu, \"workgroups\": %d, "
                 "\"balance\": %.4f}",
                 q ? ", " : "", fam_name(p.wv == 1 ? FAM_W1 : (p.wv == 2 ? FAM_W2 : (p.wv == 3 ? FAM_SN : FAM_WG))),
                 p.subs.size(),
                 p.items.size(), p.n_wg,
                 p.max_wg_cost > 0 ? p.mean_wg_cost / p.max_wg_cost : 1.0);
        js += item;
    }
    js += "], \"tuning\": [" + ctx->tune_log + "]}";
    if (js.size() + 1 > len) return fail(XENG_EINVAL, "buffer of %zu bytes too small", len);
    memcpy(buf, js.c_str(), js.size() + 1);
    return XENG_OK;
}

} // extern "C"

#include "xeng_stream.h"
#include "xeng_tune.h"
#include "xeng_tuning_file.h"
#include "xeng_ingest.h"
#include "xeng_fengine.h"
#include "xeng_static.h"
