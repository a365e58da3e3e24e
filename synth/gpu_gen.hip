// Counter-based quantised-Gaussian sample generator, GPU side.
//
// Input generation only: it stands in for the F-engine data arriving in a
// ring slot and shares nothing with the correlator. It implements the same
// definition as synth/csynth.c (which states it in full):
//   u = mix(mix(seed) + (c + 1) * 0x9E3779B97F4A7C15) >> 32,
//   c = ((t F + f) N + i) 2 + comp,
//   v = lo + #{k : u >= thr[k]}
// with mix the SplitMix64 output function, so any element drawn here equals
// the host generator's.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// number of thresholds <= u (thr non-decreasing, n_thr < 256): branch-free
// binary search over a table in LDS
__device__ __forceinline__ int level(uint32_t u, const uint32_t *thr, int n_thr)
{
    int lo = 0;
#pragma unroll
    for (int step = 128; step >= 1; step >>= 1)
        if (lo + step <= n_thr && u >= thr[lo + step - 1]) lo += step;
    return lo;
}

constexpr int GRP = 16; // inputs per thread

// Grid (ceil(n_chans * ceil(N / 16) / 256), n_time): one time sample per
// block row; each thread draws 16 consecutive inputs of one channel.
__global__ __launch_bounds__(256) void fill_kernel(uint8_t *out, int in_bits, int64_t t0,
                                                   int32_t n_chans, int32_t n_inputs,
                                                   uint64_t key, int32_t lo, int32_t n_thr,
                                                   const uint32_t *thr_base,
                                                   const uint32_t *thr_tone,
                                                   const uint8_t *tone_chan)
{
    __shared__ uint32_t s_base[256], s_tone[2][256];
    const int64_t t = blockIdx.y;
    for (int k = threadIdx.x; k < n_thr; k += blockDim.x) {
        s_base[k] = thr_base[k];
        if (thr_tone) {
            s_tone[0][k] = thr_tone[(size_t)t * 2 * n_thr + k];
            s_tone[1][k] = thr_tone[(size_t)t * 2 * n_thr + n_thr + k];
        }
    }
    __syncthreads();
    const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
    const int32_t ng = (n_inputs + GRP - 1) / GRP;
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_chans * ng) return;
    const int32_t f = w / ng;
    const int32_t i0 = (w - f * ng) * GRP;
    const bool tone = thr_tone && tone_chan && tone_chan[f];
    const uint32_t *tr = tone ? s_tone[0] : s_base;
    const uint32_t *ti = tone ? s_tone[1] : s_base;
    const uint64_t c0 = (((uint64_t)(t0 + t) * (uint64_t)n_chans + (uint64_t)f) *
                         (uint64_t)n_inputs + (uint64_t)i0) * 2u;
    uint64_t x = key + (c0 + 1u) * gamma; // element (i0, re); +gamma: im, +2 gamma: next input
    const size_t o = ((size_t)t * (size_t)n_chans + (size_t)f) * (size_t)n_inputs + (size_t)i0;
    const int n = n_inputs - i0 < GRP ? n_inputs - i0 : GRP;
    uint8_t b[2 * GRP];
#pragma unroll
    for (int r = 0; r < GRP; ++r) {
        const uint32_t ur = (uint32_t)(mix64(x) >> 32);
        const uint32_t ui = (uint32_t)(mix64(x + gamma) >> 32);
        x += 2 * gamma;
        const int vr = lo + level(ur, tr, n_thr);
        const int vi = lo + level(ui, ti, n_thr);
        if (in_bits == 4) {
            b[r] = (uint8_t)(((vr & 15) << 4) | (vi & 15));
        } else {
            b[2 * r] = (uint8_t)(int8_t)vr;
            b[2 * r + 1] = (uint8_t)(int8_t)vi;
        }
    }
    const int nb = in_bits == 4 ? n : 2 * n;
    uint8_t *dst = out + (in_bits == 4 ? o : 2 * o);
    if (nb == (in_bits == 4 ? GRP : 2 * GRP) && ((uintptr_t)dst & 15) == 0) {
        uint4 v;
        __builtin_memcpy(&v, b, 16);
        *(uint4 *)dst = v;
        if (in_bits == 8) {
            __builtin_memcpy(&v, b + 16, 16);
            *(uint4 *)(dst + 16) = v;
        }
    } else {
        for (int k = 0; k < nb; ++k) dst[k] = b[k];
    }
}

uint64_t host_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

} // namespace

extern "C" {

// Fill device buffer `out` (4-bit: uint8 [n_time][n_chans][n_inputs];
// 8-bit: int8 [...][2]) with times [t0, t0 + n_time) of the stream `seed`,
// all channels. Threshold tables are device arrays: thr_base [n_lv - 1],
// thr_tone [n_time][2][n_lv - 1] (or NULL), tone_chan [n_chans] (or NULL).
// Enqueued on `stream`; returns 0 or a hipError_t value.
int synth_fill_device(void *out, int in_bits, int64_t n_time, int64_t t0, int32_t n_chans,
                      int32_t n_inputs, uint64_t seed, int32_t lo, int32_t n_lv,
                      const uint32_t *thr_base, const uint32_t *thr_tone,
                      const uint8_t *tone_chan, void *stream)
{
    if (!out || !thr_base || n_time < 0 || n_chans < 1 || n_inputs < 1 || n_lv < 2 ||
        (in_bits != 4 && in_bits != 8))
        return (int)hipErrorInvalidValue;
    if (n_lv - 1 > 255 || (int64_t)n_chans * ((n_inputs + GRP - 1) / GRP) > (1LL << 31) - 256)
        return (int)hipErrorInvalidValue;
    const uint32_t gx = (uint32_t)(((int64_t)n_chans * ((n_inputs + GRP - 1) / GRP) + 255) / 256);
    for (int64_t ts = 0; ts < n_time; ts += 65535) {
        const uint32_t gy = (uint32_t)(n_time - ts < 65535 ? n_time - ts : 65535);
        uint8_t *o = (uint8_t *)out + (size_t)ts * (size_t)n_chans * (size_t)n_inputs * (in_bits / 4);
        const uint32_t *tt = thr_tone ? thr_tone + (size_t)ts * 2 * (n_lv - 1) : nullptr;
        hipLaunchKernelGGL(fill_kernel, dim3(gx, gy), dim3(256), 0, (hipStream_t)stream, o,
                           in_bits, t0 + ts, n_chans, n_inputs, host_mix64(seed), lo, n_lv - 1,
                           thr_base, tt, tone_chan);
    }
    return (int)hipGetLastError();
}

} // extern "C"
