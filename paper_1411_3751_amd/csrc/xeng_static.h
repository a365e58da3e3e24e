// Correlate-and-dump that allocates nothing: the persistent kernel's tile
// list lives in a file-scope device array (one copy per GPU, for as long as
// the process runs) and is rebuilt by a small kernel on every call. Part of
// the libxeng.so translation unit (included by xeng.hip after the context
// API).
#pragma once

namespace xeng {

constexpr int STATIC_MAX_ITEMS = 1 << 19;                       // tiles per call
constexpr int STATIC_MAX_WG = 4096;                              // persistent workgroups
constexpr size_t STATIC_ITEM_BYTES = (size_t)STATIC_MAX_ITEMS * sizeof(WgItem);
constexpr size_t STATIC_BYTES = STATIC_ITEM_BYTES + (size_t)(STATIC_MAX_WG + 1) * 4;

// Tile list of one subarray for the persistent kernel: tiles (channel f,
// 128-input block I, block J <= I) in locality order, the list cut into 8
// contiguous parts in proportion to the workgroups each XCD holds (workgroup
// b runs on XCD b mod 8), and each part dealt round-robin to its XCD's
// workgroups. Thread b writes workgroup b's range and tiles.
__global__ __launch_bounds__(64) void static_tiles_kernel(WgItem *__restrict__ items,
                                                          int32_t *__restrict__ wg_begin,
                                                          int32_t n_chans, int32_t nb, int32_t n_wg)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_wg) return;
    const int64_t per_chan = (int64_t)nb * (nb + 1) / 2;
    const int64_t n_items = per_chan * n_chans;
    // workgroups of XCD x: b = x, x + 8, ... < n_wg
    auto n_of = [&](int x) { return x < n_wg ? (n_wg - x + 7) / 8 : 0; };
    auto first_of = [&](int x) { // first tile of XCD x's part
        int64_t before = 0;
        for (int y = 0; y < x; ++y) before += n_of(y);
        return n_items * before / n_wg;
    };
    // tiles of workgroup c: XCD x = c % 8 deals tiles first .. last - 1 to its
    // workgroups in turn, local index w = c / 8
    auto count_of = [&](int c) {
        const int x = c & 7, w = c >> 3, nx = n_of(x);
        const int64_t len = first_of(x + 1) - first_of(x);
        return len > w ? (len - w + nx - 1) / nx : (int64_t)0;
    };
    int64_t start = 0;
    for (int c = 0; c < b; ++c) start += count_of(c);
    wg_begin[b] = (int32_t)start;
    if (b == n_wg - 1) wg_begin[n_wg] = (int32_t)(start + count_of(b));
    const int x = b & 7, w = b >> 3, nx = n_of(x);
    const int64_t f0 = first_of(x), f1 = first_of(x + 1);
    int64_t o = start;
    for (int64_t k = f0 + w; k < f1; k += nx, ++o) {
        const int64_t f = k / per_chan, t = k - f * per_chan;
        // row bi of the packed lower block triangle holding index t
        int bi = (int)((__builtin_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        if ((int64_t)bi * (bi + 1) / 2 > t) --bi;
        if ((int64_t)(bi + 1) * (bi + 2) / 2 <= t) ++bi;
        const int bj = (int)(t - (int64_t)bi * (bi + 1) / 2);
        WgItem it;
        it.cs = (uint32_t)f;
        it.ij = (uint32_t)bi | ((uint32_t)bj << 16);
        items[o] = it;
    }
}

} // namespace xeng

// The tile list's storage. Host code names it only to look up its address:
// each device's copy sits at its own address, looked up once per device.
static __device__ __align__(256) uint8_t scratch[xeng::STATIC_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES] = {};
int g_static_ncu[STATIC_MAX_DEVICES] = {};

// scratch's address and the CU count of the current device (looked up on
// the first call on that device)
int static_setup(int &dev, uint8_t *&ptr, int &n_cu)
{
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(XENG_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        int ncu = 0;
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (!p || ncu < 1) return fail(XENG_EHIP, "no scratch address or CU count on device %d", dev);
        g_static_ptr[dev] = p;
        g_static_ncu[dev] = ncu;
    }
    ptr = (uint8_t *)g_static_ptr[dev];
    n_cu = g_static_ncu[dev];
    return XENG_OK;
}

} // namespace

extern "C" {

int xeng_correlate_dump_static(const xeng_subarray *sub, const void *d_samples, void *d_out,
                               void *hip_stream)
{
    if (!sub || !d_samples || !d_out) return fail(XENG_EINVAL, "NULL argument");
    int rc = validate(*sub, 0);
    if (rc) return rc;
    if (!wave_path(*sub))
        return fail(XENG_EINVAL,
                    "the allocation-free call runs the persistent kernel only: n_inputs %d must be a "
                    "multiple of %d", sub->n_inputs, sub->in_bits == 4 ? 16 : 8);
    if (sub->n_time > xeng::SEG_T)
        return fail(XENG_EINVAL, "the allocation-free call takes at most %d samples (got %d)",
                    xeng::SEG_T, sub->n_time);
    if (((uintptr_t)d_samples & 15) != 0) return fail(XENG_EINVAL, "d_samples is not 16-byte aligned");
    if (((uintptr_t)d_out & 7) != 0) return fail(XENG_EINVAL, "d_out is not 8-byte aligned");
    const int nb = (sub->n_inputs + 127) / 128;
    const int64_t n_items = (int64_t)nb * (nb + 1) / 2 * sub->n_chans;
    if (n_items > xeng::STATIC_MAX_ITEMS)
        return fail(XENG_EINVAL,
                    "the allocation-free call takes at most %d tiles of 128 x 128 inputs per call "
                    "(n_chans * nb (nb + 1) / 2 with nb = ceil(N / 128)); this shape has %lld",
                    xeng::STATIC_MAX_ITEMS, (long long)n_items);
    int dev = 0, n_cu = 0;
    uint8_t *ptr = nullptr;
    rc = static_setup(dev, ptr, n_cu);
    if (rc) return rc;
    const int n_wg = (int)std::min<int64_t>(std::min<int64_t>((int64_t)n_cu * WG_PER_CU, n_items),
                                            xeng::STATIC_MAX_WG);
    hipStream_t st = (hipStream_t)hip_stream;
    xeng::WgItem *items = (xeng::WgItem *)ptr;
    int32_t *wg_begin = (int32_t *)(ptr + xeng::STATIC_ITEM_BYTES);
    hipLaunchKernelGGL(xeng::static_tiles_kernel, dim3((n_wg + 63) / 64), dim3(64), 0, st, items,
                       wg_begin, sub->n_chans, nb, n_wg);
    HIP_TRY(hipGetLastError());
    xeng::WgArgs a;
    memset(&a, 0, sizeof a);
    xeng::WgSub &w = a.subs[0];
    w.samples = (const uint8_t *)d_samples;
    w.src = nullptr; // one segment: nothing to add
    w.dst = (int32_t *)d_out;
    w.t_begin = 0;
    w.t_count = sub->n_time;
    w.n_chans = sub->n_chans;
    w.n_inputs = sub->n_inputs;
    a.items = items;
    a.wg_begin = wg_begin;
    const dim3 g(n_wg), b(xeng::WG_THREADS);
    if (sub->engine == XENG_ENGINE_FP8)
        hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_F8, 4, true>), g, b, 0, st, a);
    else if (sub->in_bits == 4)
        hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 4, true>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((xeng::xcorr_wg_kernel<xeng::ENG_I8, 8, true>), g, b, 0, st, a);
    HIP_TRY(hipGetLastError());
    return XENG_OK;
}

} // extern "C"
