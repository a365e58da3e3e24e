// Packet ingest: corner turn of F-engine packets into a gulp buffer, with
// accounting of missing, duplicate and rejected packets. Part of the
// libxeng.so translation unit (included by xeng.hip). The packet format is
// declared in include/xeng.h.
//
// Kernels (all on the caller's stream):
//   ingest_clear_kernel   set every block's owner to "none", zero the counters
//   ingest_claim_kernel   one wave per packet: validate the header and claim
//                         the packet's block with an atomic minimum of the
//                         packet index (the first copy in buffer order owns
//                         the block, whatever order the waves run in)
//   ingest_scatter_kernel one wave per packet: count it (received, duplicate
//                         or rejected) and, if it owns its block, copy the
//                         payload rows to [time][chan][input] in 16-, 4- or
//                         1-byte units
//   ingest_fill_kernel    one wave per 64 expected blocks: zero-fill the
//                         blocks nobody owns and count them
#pragma once

namespace xeng {

struct IngestGeom {
    int64_t gulp_t0;
    int32_t n_time, n_chans, n_inputs, bps;     // gulp shape, bytes per sample
    int32_t pt, pc, pi;                         // packet block shape
    int32_t nb_t, nb_f, nb_i;                   // blocks per gulp dimension
    int32_t unit;                               // copy unit in bytes (16, 4 or 1)
    int64_t stride;                             // bytes between packets
};

enum { CNT_RECEIVED = 0, CNT_MISSING = 1, CNT_DUPLICATE = 2, CNT_REJECTED = 3 };

// The counters are spread over CNT_SLOTS copies, one 128-byte line each, and
// summed on the host: one packet per wave adds to them, and a single address
// would serialise every one of those atomics in one L2 channel.
constexpr int CNT_SLOTS = 64;
constexpr int CNT_STRIDE = 16; // counters per slot line (4 used)

__device__ __forceinline__ unsigned long long *cnt_slot(unsigned long long *counts, int64_t wave)
{
    return counts + (size_t)(wave & (CNT_SLOTS - 1)) * CNT_STRIDE;
}

constexpr uint32_t NO_OWNER = 0xFFFFFFFFu;

__global__ void ingest_clear_kernel(uint32_t *owner, int64_t n_blocks, unsigned long long *counts)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_blocks;
         k += (int64_t)gridDim.x * blockDim.x)
        owner[k] = NO_OWNER;
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < CNT_SLOTS * 4; k += blockDim.x)
            counts[(size_t)(k >> 2) * CNT_STRIDE + (k & 3)] = 0ull;
}

// The block a packet's header names within the gulp, or -1 if the packet is
// rejected (bad magic, not aligned to the blocks, or outside the gulp).
// Every lane reads the same 16 header bytes.
__device__ __forceinline__ int64_t packet_block(const uint8_t *pk, const IngestGeom &g,
                                                int64_t &dt, int64_t &chan0, int64_t &input0)
{
    const uint64_t t0 = *(const uint64_t *)pk;
    const uint32_t ci = *(const uint32_t *)(pk + 8);
    const uint32_t magic = *(const uint32_t *)(pk + 12);
    chan0 = ci & 0xFFFFu;
    input0 = ci >> 16;
    dt = (int64_t)t0 - g.gulp_t0;
    const bool ok = magic == XENG_PACKET_MAGIC && dt >= 0 && dt < g.n_time && dt % g.pt == 0 &&
                    chan0 < g.n_chans && chan0 % g.pc == 0 && input0 < g.n_inputs &&
                    input0 % g.pi == 0;
    return ok ? ((dt / g.pt) * g.nb_f + chan0 / g.pc) * g.nb_i + input0 / g.pi : -1;
}

__global__ __launch_bounds__(256) void ingest_claim_kernel(const uint8_t *__restrict__ pkts,
                                                           int64_t n_packets, IngestGeom g,
                                                           uint32_t *owner)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n_packets;
         p += waves) {
        int64_t dt, chan0, input0;
        const int64_t b = packet_block(pkts + p * g.stride, g, dt, chan0, input0);
        if (b >= 0 && lane == 0) atomicMin(&owner[b], (uint32_t)p);
    }
}

template <int UNIT>
__device__ __forceinline__ void copy_unit(uint8_t *dst, const uint8_t *src)
{
    if constexpr (UNIT == 16) *(uint4 *)dst = *(const uint4 *)src;
    else if constexpr (UNIT == 4) *(uint32_t *)dst = *(const uint32_t *)src;
    else *dst = *src;
}

// destination of unit u of a block (t, chan, input) in the gulp: row = (pt,
// pc) of the block, w = unit within the row (all indices of one block fit
// int32: a block is at most a packet's payload)
__device__ __forceinline__ uint8_t *block_unit(uint8_t *gulp, const IngestGeom &g, int64_t t0,
                                               int64_t chan0, int64_t input0, int32_t u,
                                               int32_t units_row, int32_t unit)
{
    const int32_t row = u / units_row, w = u - row * units_row;
    const int32_t pt = row / g.pc, pc = row - pt * g.pc;
    return gulp + (((t0 + pt) * g.n_chans + chan0 + pc) * g.n_inputs + input0) * g.bps +
           (int64_t)w * unit;
}

template <int UNIT>
__global__ __launch_bounds__(256) void ingest_scatter_kernel(const uint8_t *__restrict__ pkts,
                                                             int64_t n_packets, IngestGeom g,
                                                             uint8_t *__restrict__ gulp,
                                                             const uint32_t *owner,
                                                             unsigned long long *counts)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int32_t units_row = g.pi * g.bps / UNIT;
    const int32_t units = units_row * g.pt * g.pc;
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n_packets;
         p += waves) {
        const uint8_t *pk = pkts + p * g.stride;
        int64_t dt, chan0, input0;
        const int64_t b = packet_block(pk, g, dt, chan0, input0);
        // 0 rejected, 1 owner of its block, 2 a later copy of a claimed block
        const int claim = b < 0 ? 0 : (owner[b] == (uint32_t)p ? 1 : 2);
        if (lane == 0)
            atomicAdd(&cnt_slot(counts, p)[claim == 1 ? CNT_RECEIVED : claim == 2 ? CNT_DUPLICATE
                                                                               : CNT_REJECTED],
                      1ull);
        if (claim != 1) continue;
        const uint8_t *src = pk + 16;
        for (int32_t u = lane; u < units; u += 64)
            copy_unit<UNIT>(block_unit(gulp, g, dt, chan0, input0, u, units_row, UNIT),
                            src + (int64_t)u * UNIT);
    }
}

// one wave per 64 consecutive expected blocks: a ballot over their owners
// finds the missing ones (most are present), which the wave then zero-fills
// one after the other; one count per wave
template <int UNIT>
__global__ __launch_bounds__(256) void ingest_fill_kernel(IngestGeom g, uint8_t *__restrict__ gulp,
                                                          const uint32_t *owner,
                                                          unsigned long long *counts)
{
    const int lane = threadIdx.x & 63;
    const int64_t n_blocks = (int64_t)g.nb_t * g.nb_f * g.nb_i;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int32_t units_row = g.pi * g.bps / UNIT;
    const int32_t units = units_row * g.pt * g.pc;
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w * 64 < n_blocks;
         w += waves) {
        const int64_t b = w * 64 + lane;
        const bool missing = b < n_blocks && owner[b] == NO_OWNER;
        uint64_t todo = __ballot(missing);
        if (lane == 0 && todo) atomicAdd(&cnt_slot(counts, w)[CNT_MISSING], (unsigned long long)__popcll(todo));
        while (todo) {
            const int64_t bm = w * 64 + __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t ib = bm % g.nb_i, fb = (bm / g.nb_i) % g.nb_f, tb = bm / ((int64_t)g.nb_i * g.nb_f);
            for (int32_t u = lane; u < units; u += 64) {
                uint8_t *dst = block_unit(gulp, g, tb * g.pt, fb * g.pc, ib * g.pi, u, units_row, UNIT);
                if constexpr (UNIT == 16) *(uint4 *)dst = make_uint4(0u, 0u, 0u, 0u);
                else if constexpr (UNIT == 4) *(uint32_t *)dst = 0u;
                else *dst = 0;
            }
        }
    }
}

} // namespace xeng

struct xeng_ingest {
    xeng::IngestGeom g{};
    int64_t n_blocks = 0;
    uint32_t *d_owner = nullptr;        // per block: index of the packet that fills it
    unsigned long long *d_counts = nullptr;
    hipStream_t last = nullptr;         // stream of the last gulp
    hipEvent_t last_done = nullptr;     // recorded after the last gulp's kernels
    bool used = false;
};

extern "C" {

int xeng_ingest_create(const xeng_subarray *sub, const xeng_packet_format *fmt, xeng_ingest **out)
{
    if (!out) return fail(XENG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sub || !fmt) return fail(XENG_EINVAL, "NULL argument");
    int rc = validate(*sub, 0);
    if (rc) return rc;
    if (fmt->pkt_time < 1 || fmt->pkt_chans < 1 || fmt->pkt_inputs < 1)
        return fail(XENG_EINVAL, "packet block sizes must be >= 1");
    if (sub->n_time % fmt->pkt_time || sub->n_chans % fmt->pkt_chans ||
        sub->n_inputs % fmt->pkt_inputs)
        return fail(XENG_EINVAL, "packet blocks (%d, %d, %d) do not divide the gulp (%d, %d, %d)",
                    fmt->pkt_time, fmt->pkt_chans, fmt->pkt_inputs, sub->n_time, sub->n_chans,
                    sub->n_inputs);
    if (sub->n_chans > 65535 || sub->n_inputs > 65535)
        return fail(XENG_EINVAL, "the packet header holds 16-bit channel and input indices");
    xeng_ingest *ig = new (std::nothrow) xeng_ingest;
    if (!ig) return fail(XENG_ENOMEM, "host allocation failed");
    xeng::IngestGeom &g = ig->g;
    g.n_time = sub->n_time;
    g.n_chans = sub->n_chans;
    g.n_inputs = sub->n_inputs;
    g.bps = sub->in_bits / 4;
    g.pt = fmt->pkt_time;
    g.pc = fmt->pkt_chans;
    g.pi = fmt->pkt_inputs;
    g.nb_t = sub->n_time / g.pt;
    g.nb_f = sub->n_chans / g.pc;
    g.nb_i = sub->n_inputs / g.pi;
    const int64_t payload = (int64_t)g.pt * g.pc * g.pi * g.bps;
    g.stride = 16 + (payload + 15) / 16 * 16;
    // copy unit: every row start and length in both buffers is a multiple of it
    const int64_t row = (int64_t)g.pi * g.bps, gstride = (int64_t)g.n_inputs * g.bps;
    g.unit = (row % 16 == 0 && gstride % 16 == 0) ? 16 : (row % 4 == 0 && gstride % 4 == 0) ? 4 : 1;
    ig->n_blocks = (int64_t)g.nb_t * g.nb_f * g.nb_i;
    hipError_t e = hipMalloc((void **)&ig->d_owner, sizeof(uint32_t) * (size_t)ig->n_blocks);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ig->d_counts,
                      (size_t)xeng::CNT_SLOTS * xeng::CNT_STRIDE * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ig->last_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (ig->d_owner) (void)hipFree(ig->d_owner);
        if (ig->d_counts) (void)hipFree(ig->d_counts);
        delete ig;
        return fail(XENG_ENOMEM, "hipMalloc for the ingest block owners: %s", hipGetErrorString(e));
    }
    *out = ig;
    return XENG_OK;
}

int xeng_ingest_packet_stride(const xeng_ingest *ig, int64_t *out)
{
    if (!ig || !out) return fail(XENG_EINVAL, "NULL argument");
    *out = ig->g.stride;
    return XENG_OK;
}

int xeng_ingest_gulp(xeng_ingest *ig, const void *d_packets, int64_t n_packets, int64_t gulp_t0,
                     void *d_gulp, void *hip_stream)
{
    if (!ig || !d_gulp) return fail(XENG_EINVAL, "NULL argument");
    if (n_packets < 0 || (n_packets > 0 && !d_packets)) return fail(XENG_EINVAL, "bad packet buffer");
    if (((uintptr_t)d_packets & 15) || ((uintptr_t)d_gulp & 15))
        return fail(XENG_EINVAL, "packet and gulp buffers must be 16-byte aligned");
    if (n_packets >= (int64_t)xeng::NO_OWNER)
        return fail(XENG_EINVAL, "at most %u packets per gulp", xeng::NO_OWNER - 1);
    hipStream_t st = (hipStream_t)hip_stream;
    // the engine's owner table and counters are reused: a gulp on another
    // stream waits for the previous gulp's kernels
    if (ig->used && st != ig->last) HIP_TRY(hipStreamWaitEvent(st, ig->last_done, 0));
    xeng::IngestGeom g = ig->g;
    g.gulp_t0 = gulp_t0;
    const int cb = (int)std::min<int64_t>((ig->n_blocks + 255) / 256, 1024);
    hipLaunchKernelGGL(xeng::ingest_clear_kernel, dim3(cb < 1 ? 1 : cb), dim3(256), 0, st,
                       ig->d_owner, ig->n_blocks, ig->d_counts);
    HIP_TRY(hipGetLastError());
    if (n_packets > 0) {
        const unsigned sb = (unsigned)std::min<int64_t>((n_packets + 3) / 4, 65536);
        const uint8_t *pk = (const uint8_t *)d_packets;
        uint8_t *gp = (uint8_t *)d_gulp;
        hipLaunchKernelGGL(xeng::ingest_claim_kernel, dim3(sb), dim3(256), 0, st, pk, n_packets, g,
                           ig->d_owner);
        HIP_TRY(hipGetLastError());
        if (g.unit == 16)
            hipLaunchKernelGGL(xeng::ingest_scatter_kernel<16>, dim3(sb), dim3(256), 0, st, pk,
                               n_packets, g, gp, ig->d_owner, ig->d_counts);
        else if (g.unit == 4)
            hipLaunchKernelGGL(xeng::ingest_scatter_kernel<4>, dim3(sb), dim3(256), 0, st, pk,
                               n_packets, g, gp, ig->d_owner, ig->d_counts);
        else
            hipLaunchKernelGGL(xeng::ingest_scatter_kernel<1>, dim3(sb), dim3(256), 0, st, pk,
                               n_packets, g, gp, ig->d_owner, ig->d_counts);
        HIP_TRY(hipGetLastError());
    }
    const unsigned fb = (unsigned)std::min<int64_t>((ig->n_blocks + 255) / 256, 65536);
    if (g.unit == 16)
        hipLaunchKernelGGL(xeng::ingest_fill_kernel<16>, dim3(fb < 1 ? 1 : fb), dim3(256), 0, st, g,
                           (uint8_t *)d_gulp, ig->d_owner, ig->d_counts);
    else if (g.unit == 4)
        hipLaunchKernelGGL(xeng::ingest_fill_kernel<4>, dim3(fb < 1 ? 1 : fb), dim3(256), 0, st, g,
                           (uint8_t *)d_gulp, ig->d_owner, ig->d_counts);
    else
        hipLaunchKernelGGL(xeng::ingest_fill_kernel<1>, dim3(fb < 1 ? 1 : fb), dim3(256), 0, st, g,
                           (uint8_t *)d_gulp, ig->d_owner, ig->d_counts);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ig->last_done, st));
    ig->last = st;
    ig->used = true;
    return XENG_OK;
}

int xeng_ingest_stats_get(xeng_ingest *ig, xeng_ingest_stats *out)
{
    if (!ig || !out) return fail(XENG_EINVAL, "NULL argument");
    HIP_TRY(hipEventSynchronize(ig->last_done));
    unsigned long long slots[xeng::CNT_SLOTS * xeng::CNT_STRIDE];
    HIP_TRY(hipMemcpy(slots, ig->d_counts, sizeof slots, hipMemcpyDeviceToHost));
    unsigned long long c[4] = {0ull, 0ull, 0ull, 0ull};
    for (int k = 0; k < xeng::CNT_SLOTS; ++k)
        for (int j = 0; j < 4; ++j) c[j] += slots[k * xeng::CNT_STRIDE + j];
    out->received = (int64_t)c[xeng::CNT_RECEIVED];
    out->missing = (int64_t)c[xeng::CNT_MISSING];
    out->duplicate = (int64_t)c[xeng::CNT_DUPLICATE];
    out->rejected = (int64_t)c[xeng::CNT_REJECTED];
    return XENG_OK;
}

int xeng_ingest_destroy(xeng_ingest *ig)
{
    if (!ig) return XENG_OK;
    (void)hipStreamSynchronize(ig->last);
    if (ig->d_owner) (void)hipFree(ig->d_owner);
    if (ig->d_counts) (void)hipFree(ig->d_counts);
    if (ig->last_done) (void)hipEventDestroy(ig->last_done);
    delete ig;
    return XENG_OK;
}

} // extern "C"
