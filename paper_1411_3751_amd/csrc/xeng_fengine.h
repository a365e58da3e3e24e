// F-engine: polyphase filter bank, FFT and requantisation to 4+4 bits
// (Section 2.2: a 4-tap, 8192-point PFB made of an FIR filter with a Hamming
// window and 18-bit coefficients followed by an FFT whose stages halve the
// data, 24.0 kHz channels; one band-average digital gain; requantisation of
// the 18+18-bit values to 4+4 bits; a contiguous group of channels selected).
// Part of the libxeng.so translation unit (included by xeng.hip).
//
// Definition computed (spectrum m of input n, k < P = 8192, L = 4 P):
//   c[l]  = clip(rint(2^17 w[l] sinc((l - (L-1)/2) / P)), -2^17, 2^17 - 1),
//           w the symmetric Hamming window of length L
//   y[k]  = sum_tap c[tap P + k] x[(m + tap) P + k]          (exact, int32)
//   Y[ch] = gain 2^-17 / P sum_k y[k] exp(-2 pi i k ch / P)    (fp32)
//   code  = clip(rint(Re Y), -8, 7) << 4 | clip(rint(Im Y), -8, 7) (nibbles)
// written to out[m][ch - chan0][n], the X-engine's [time][channel][input].
//
// One workgroup of 256 threads takes one spectrum of G <= 4 consecutive
// inputs, one input after the other; LDS holds the FFT buffer (35 KB) and the
// pass-twiddle tables (4.6 KB), registers stay under 128, so four workgroups
// share a CU:
//   * FIR, exact in int32: thread t owns samples [16t, 16t+16) and their
//     mirror [P-16t-16, P-16t) of each tap block. The prototype is
//     symmetric (c[l] = c[4P-1-l]), so taps 2 and 3 at a position are taps
//     1 and 0 at its mirror: only taps 0 and 1 are loaded. z[j] = y[2j] +
//     i y[2j+1] goes to LDS;
//   * the P-point real FFT as a 4096-point complex FFT of z: three radix-16
//     Stockham passes, 16 points per thread, through one padded LDS buffer
//     (index i at i + i/16 keeps the strided accesses conflict-free);
//   * real-FFT split Y[c] = (Z[c] + conj Z[H-c]) / 2 - i exp(-2 pi i c / P)
//     (Z[c] - conj Z[H-c]) / 2 for the selected channels, requantised;
//     thread t keeps the codes of channels chan0 + t + 256 k in register k,
//     one byte per input, and stores them as one G-byte word per channel.
// Workgroups are numbered so that the consecutive ones each XCD runs hold
// consecutive inputs of one spectrum, so partial output lines meet in that
// XCD's L2.
#pragma once

namespace xeng {

constexpr int FE_P = 8192;                 // FFT points (real samples per spectrum)
constexpr int FE_H = FE_P / 2;             // complex FFT points
constexpr int FE_TAPS = 4;
constexpr int FE_THREADS = 256;            // = FE_H / 16 radix-16 butterflies
constexpr int FE_LDS = FE_H + FE_H / 16;   // padded complex slots
constexpr int FE_MAX_GROUP = 4;
// pass twiddle rows of 16 (r < 16): row j < 16 holds exp(-2 pi i j r / 4096),
// row 16 + i holds exp(-2 pi i i r / 256). Pass 2 of thread t uses row
// 16 + t%16; pass 3 uses exp(-2 pi i t r / 4096), the product of rows t%16
// and 16 + t/16.
constexpr int FE_TW_ROWS = 32;
constexpr int FE_TW_LDS_ROW = 18;          // LDS row stride in complex values (bank spread)

// exp(-2 pi i k / 32), k < 16: steps between the channels of one thread
__device__ constexpr float FE_W32[16][2] = {
    {1.000000000e+00f, 0.f}, {9.807852804e-01f, -1.950903220e-01f},
    {9.238795325e-01f, -3.826834324e-01f}, {8.314696123e-01f, -5.555702330e-01f},
    {7.071067812e-01f, -7.071067812e-01f}, {5.555702330e-01f, -8.314696123e-01f},
    {3.826834324e-01f, -9.238795325e-01f}, {1.950903220e-01f, -9.807852804e-01f},
    {0.f, -1.000000000e+00f}, {-1.950903220e-01f, -9.807852804e-01f},
    {-3.826834324e-01f, -9.238795325e-01f}, {-5.555702330e-01f, -8.314696123e-01f},
    {-7.071067812e-01f, -7.071067812e-01f}, {-8.314696123e-01f, -5.555702330e-01f},
    {-9.238795325e-01f, -3.826834324e-01f}, {-9.807852804e-01f, -1.950903220e-01f}};

struct FeArgs {
    const int8_t *adc;     // [N][stride] ADC samples
    int64_t adc_stride;
    const int32_t *coef;   // [taps P] 18-bit coefficients
    const float2 *tw;      // [FE_TW_ROWS][16] pass twiddles, rows described at FE_TW_ROWS
    const float2 *tw_r;    // [FE_H] exp(-2 pi i c / FE_P)
    uint8_t *out;          // [n_spectra][n_chans][N]
    float2 *spec;          // optional [n_spectra][n_chans][N] scaled values, or null
    int32_t n_inputs, n_chans, chan0, group;
    int32_t n_groups;      // n_inputs / group
    int32_t n_blocks;      // n_spectra * n_groups
    float scale;           // gain 2^-17 / P
};

__device__ __forceinline__ int fe_pad(int i) { return i + (i >> 4); }

// the 16 twiddles of LDS row `row`
__device__ __forceinline__ void fe_twiddle_row(const float2 *twl, int row, float2 (&w)[16])
{
    const float4 *p = (const float4 *)(twl + row * FE_TW_LDS_ROW);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float4 q = p[k];
        w[2 * k] = make_float2(q.x, q.y);
        w[2 * k + 1] = make_float2(q.z, q.w);
    }
}

__device__ __forceinline__ float2 fe_cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// a * exp(-2 pi i e / 16) for a compile-time e
template <int E>
__device__ __forceinline__ float2 fe_w16(float2 a)
{
    constexpr float C1 = 0.92387953251128674f, S1 = 0.38268343236508978f, R = 0.70710678118654752f;
    constexpr int e = E & 15;
    if constexpr (e == 0) return a;
    else if constexpr (e == 4) return make_float2(a.y, -a.x);
    else if constexpr (e == 8) return make_float2(-a.x, -a.y);
    else if constexpr (e == 12) return make_float2(-a.y, a.x);
    else if constexpr (e == 2) return make_float2(R * (a.x + a.y), R * (a.y - a.x));
    else if constexpr (e == 6) return make_float2(R * (a.y - a.x), -R * (a.x + a.y));
    else {
        // (c, s) = (cos, sin)(2 pi e / 16) from the first-octant values
        constexpr float c = (e == 1 || e == 15) ? C1 : (e == 3 || e == 13) ? S1
                          : (e == 5 || e == 11) ? -S1 : (e == 7 || e == 9) ? -C1
                          : (e == 10) ? -R : (e == 14) ? R : 0.f;
        constexpr float s = (e == 1 || e == 7) ? S1 : (e == 3 || e == 5) ? C1
                          : (e == 9 || e == 15) ? -S1 : (e == 11 || e == 13) ? -C1
                          : (e == 10) ? -R : (e == 14) ? -R : 0.f;
        // multiply by (c - i s)
        return make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
    }
}

// in-place 4-point DFT, X[k] = sum_n a[n] exp(-2 pi i n k / 4)
__device__ __forceinline__ void fe_dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    const float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
    const float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
    const float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
    const float2 t3 = make_float2(a1.y - a3.y, a3.x - a1.x);  // -i (a1 - a3)
    a0 = make_float2(t0.x + t2.x, t0.y + t2.y);
    a2 = make_float2(t0.x - t2.x, t0.y - t2.y);
    a1 = make_float2(t1.x + t3.x, t1.y + t3.y);
    a3 = make_float2(t1.x - t3.x, t1.y - t3.y);
}

template <int K1, int N2>
__device__ __forceinline__ void fe_tw_inner(float2 (&v)[16])
{
    v[4 * K1 + N2] = fe_w16<K1 * N2>(v[4 * K1 + N2]);
}

// 16-point DFT, natural order in and out: n = 4 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void fe_dft16(float2 (&v)[16])
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) fe_dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] now holds the n1-transform; twiddle exp(-2 pi i n2 k1 / 16)
    fe_tw_inner<1, 1>(v); fe_tw_inner<1, 2>(v); fe_tw_inner<1, 3>(v);
    fe_tw_inner<2, 1>(v); fe_tw_inner<2, 2>(v); fe_tw_inner<2, 3>(v);
    fe_tw_inner<3, 1>(v); fe_tw_inner<3, 2>(v); fe_tw_inner<3, 3>(v);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) fe_dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] = X[k1 + 4 k2]: reorder
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[k];
}

__global__ __launch_bounds__(FE_THREADS, 4) void fengine_kernel(FeArgs a)
{
    __shared__ float2 z[FE_LDS];
    __shared__ __align__(16) float2 twl[FE_TW_ROWS * FE_TW_LDS_ROW];
    const int t = threadIdx.x;

    // workgroup number -> (spectrum, input group); the dispatcher deals
    // workgroups round-robin over 8 XCDs, so hand each XCD a contiguous range
    const int b = blockIdx.x, nb = a.n_blocks;
    const int xcd = b & 7, q8 = nb >> 3, r8 = nb & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int64_t m = logical / a.n_groups;
    const int n0 = (logical - (int)m * a.n_groups) * a.group;

    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)a.coef, (short)0, FE_TAPS * FE_P * 4, 0x00020000);
    // pass twiddle table into LDS (32 rows of 16, padded rows)
    for (int i = t; i < FE_TW_ROWS * 16; i += FE_THREADS)
        twl[(i >> 4) * FE_TW_LDS_ROW + (i & 15)] = a.tw[i];
    // this thread's first channel twiddle exp(-2 pi i (chan0 + t) / P); the
    // others follow by steps of exp(-2 pi i 256 / P) = exp(-2 pi i / 32)
    const float hs = 0.5f * a.scale;
    const float2 wr0 = a.tw_r[(a.chan0 + t) & (FE_H - 1)];
    const float2 wc0 = make_float2(hs * wr0.x, hs * wr0.y);

    uint32_t cw[FE_H / FE_THREADS];
#pragma unroll
    for (int k = 0; k < FE_H / FE_THREADS; ++k) cw[k] = 0;
    __syncthreads();

    for (int g = 0; g < a.group; ++g) {
        // per-thread indices recomputed each input (not held in registers across it)
        int tt = t;
        asm volatile("" : "+v"(tt));
        const int n = n0 + g;
        float2 v[16];
        // FIR. Thread tt takes positions A = [16 tt, 16 tt + 16) and their
        // mirror A' = [P - 16 tt - 16, P - 16 tt) of every tap block (complex
        // points 8 tt + e and H - 8 tt - 8 + e, e < 8). The prototype is
        // symmetric, c[l] = c[4P - 1 - l], so taps 2 and 3 at a position are
        // taps 1 and 0 at its mirror: loading taps 0 and 1 over A and A' gives
        // all four.
        {
            const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.adc + (int64_t)n * a.adc_stride + m * FE_P), (short)0, FE_TAPS * FE_P, 0x00020000);
            const int oa = 16 * tt, ob = FE_P - 16 * tt - 16;
            uint32_t xs[FE_TAPS][2][4];
#pragma unroll
            for (int tap = 0; tap < FE_TAPS; ++tap)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rx, h ? ob : oa, tap * FE_P, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) xs[tap][h][q] = w[q];
                }
            // Two halves, each needing 32 coefficients: half s takes A positions
            // [8s, 8s+8) and A' positions [8(1-s), 8(1-s)+8), whose mirrors are
            // each other's. cA = taps 0, 1 at A + 8s; cB = taps 0, 1 at A' + 8(1-s).
            auto xb = [&](int tap, int h, int i) { return (int)(int8_t)(xs[tap][h][i >> 2] >> (8 * (i & 3))); };
#pragma unroll
            for (int hs = 0; hs < 2; ++hs) {
                const int sa = 8 * hs, sb = 8 - 8 * hs;
                uint32_t cA[2][8], cB[2][8];
#pragma unroll
                for (int tap = 0; tap < 2; ++tap)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const auto wa = __builtin_amdgcn_raw_buffer_load_b128(rc, 4 * (oa + sa) + 16 * q,
                                                                              4 * FE_P * tap, 0);
                        const auto wb = __builtin_amdgcn_raw_buffer_load_b128(rc, 4 * (ob + sb) + 16 * q,
                                                                              4 * FE_P * tap, 0);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            cA[tap][4 * q + e] = wa[e];
                            cB[tap][4 * q + e] = wb[e];
                        }
                    }
                int acc[2][8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    // A position i = sa + j; its mirror 15 - i = sb + 7 - j in A'
                    const int i = sa + j;
                    acc[0][j] = __mul24((int)cA[0][j], xb(0, 0, i)) + __mul24((int)cA[1][j], xb(1, 0, i)) +
                                __mul24((int)cB[1][7 - j], xb(2, 0, i)) + __mul24((int)cB[0][7 - j], xb(3, 0, i));
                    // A' position i' = sb + j; its mirror 15 - i' = sa + 7 - j in A
                    const int ib = sb + j;
                    acc[1][j] = __mul24((int)cB[0][j], xb(0, 1, ib)) + __mul24((int)cB[1][j], xb(1, 1, ib)) +
                                 __mul24((int)cA[1][7 - j], xb(2, 1, ib)) + __mul24((int)cA[0][7 - j], xb(3, 1, ib));
                }
                // complex points 8 tt + sa/2 + e and H - 8 tt - 8 + sb/2 + e, e < 4
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    z[fe_pad(8 * tt + sa / 2 + e)] = make_float2((float)acc[0][2 * e], (float)acc[0][2 * e + 1]);
                    z[fe_pad(FE_H - 8 * tt - 8 + sb / 2 + e)] =
                        make_float2((float)acc[1][2 * e], (float)acc[1][2 * e + 1]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();
        // pass 1 (span 1): points tt + 256 r, no twiddles; output index 16 tt + r
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = z[fe_pad(tt + 256 * r)];
        fe_dft16(v);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) z[fe_pad(16 * tt + r)] = v[r];
        __syncthreads();
        // pass 2 (span 16), twiddles exp(-2 pi i (tt%16) r / 256)
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = z[fe_pad(tt + 256 * r)];
        {
            float2 w[16];
            fe_twiddle_row(twl, 16 + (tt & 15), w);
#pragma unroll
            for (int r = 1; r < 16; ++r) v[r] = fe_cmul(v[r], w[r]);
        }
        fe_dft16(v);
        __syncthreads();
        {
            const int base = (tt >> 4) * 256 + (tt & 15);
#pragma unroll
            for (int r = 0; r < 16; ++r) z[fe_pad(base + 16 * r)] = v[r];
        }
        __syncthreads();
        // pass 3 (span 256), twiddles exp(-2 pi i tt r / 4096); output in
        // natural order, Z[tt + 256 r]
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = z[fe_pad(tt + 256 * r)];
        {
            // exp(-2 pi i tt r / 4096) = row tt%16 times row 16 + tt/16, applied in turn
            float2 w[16];
            fe_twiddle_row(twl, tt & 15, w);
#pragma unroll
            for (int r = 1; r < 16; ++r) v[r] = fe_cmul(v[r], w[r]);
            fe_twiddle_row(twl, 16 + (tt >> 4), w);
#pragma unroll
            for (int r = 1; r < 16; ++r) v[r] = fe_cmul(v[r], w[r]);
        }
        fe_dft16(v);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) z[fe_pad(tt + 256 * r)] = v[r];
        __syncthreads();
        // real-FFT split, gain, requantisation of the selected channels;
        // thread tt keeps the codes of channels c0 + 256 k in register k.
        {
            const int c0 = a.chan0 + tt;
            // z index of channel c0 + 256 k is pad(c0) + 272 k; of H - c0 - 256 k
            // it is pad(H - c0) - 272 k (channel 0 pairs with itself)
            const int pc0 = fe_pad(c0), pn0 = fe_pad(FE_H - c0);
            // the channel twiddles (already times the scale) are rebuilt from
            // wc0 for every input rather than held in sixteen register pairs
            float2 wc = wc0;
            asm volatile("" : "+v"(wc.x), "+v"(wc.y));
#pragma unroll
            for (int k = 0; k < FE_H / FE_THREADS; ++k) {
                const int q = tt + FE_THREADS * k;
                if (q < a.n_chans) {
                    const float2 zc = z[pc0 + 272 * k];
                    const float2 zn = z[(k == 0 && c0 == 0) ? 0 : pn0 - 272 * k];
                    const float ex = zc.x + zn.x, ey = zc.y - zn.y;        // 2 E
                    const float2 d = make_float2(zc.x - zn.x, zc.y + zn.y); // 2 D
                    const float2 wk = k ? fe_cmul(wc, make_float2(FE_W32[k][0], FE_W32[k][1])) : wc;
                    const float2 wd = fe_cmul(wk, d);
                    // Y = s (E - i W D) with s = scale / 2 (the halves of E and D)
                    const float yr = __builtin_fmaf(hs, ex, wd.y);
                    const float yi = __builtin_fmaf(hs, ey, -wd.x);
                    if (a.spec)
                        a.spec[((int64_t)m * a.n_chans + q) * a.n_inputs + n] = make_float2(yr, yi);
                    // round half to even and clip to [-8, 7]: adding 1.5 * 2^23
                    // leaves round(y) in the low mantissa bits (|y| < 2^22), the
                    // clip is an integer clamp on those bits, whose low nibble
                    // is then the two's complement code
                    constexpr int MAGIC = 0x4B400000;
                    const int br = __builtin_bit_cast(int, yr + 12582912.0f);
                    const int bi = __builtin_bit_cast(int, yi + 12582912.0f);
                    const uint32_t qr = (uint32_t)min(max(br, MAGIC - 8), MAGIC + 7);
                    const uint32_t qi = (uint32_t)min(max(bi, MAGIC - 8), MAGIC + 7);
                    cw[k] |= (((qr << 4) & 0xF0u) | (qi & 15u)) << (8 * g);
                }
            }
        }
        __syncthreads();
    }

    // one G-byte store per channel
    uint8_t *o = a.out + (int64_t)m * a.n_chans * a.n_inputs + n0;
#pragma unroll
    for (int k = 0; k < FE_H / FE_THREADS; ++k) {
        const int q = t + FE_THREADS * k;
        if (q < a.n_chans) {
            uint8_t *d = o + (int64_t)q * a.n_inputs;
            if (a.group == 4) *(uint32_t *)d = cw[k];
            else if (a.group == 2) *(uint16_t *)d = (uint16_t)cw[k];
            else d[0] = (uint8_t)cw[k];
        }
    }
}

} // namespace xeng

struct xeng_fengine {
    xeng_fengine_config cfg{};
    int group = 1;
    int32_t *d_coef = nullptr;
    float2 *d_tw = nullptr, *d_twr = nullptr;
};

extern "C" {

int xeng_fengine_create(const xeng_fengine_config *cfg, xeng_fengine **out)
{
    using namespace xeng;
    if (!out) return fail(XENG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(XENG_EINVAL, "cfg is NULL");
    if (cfg->n_inputs < 1 || cfg->n_inputs > 65535)
        return fail(XENG_EINVAL, "n_inputs %d out of [1, 65535]", cfg->n_inputs);
    if (cfg->n_chans < 1 || cfg->chan0 < 0 || cfg->chan0 + cfg->n_chans > FE_H)
        return fail(XENG_EINVAL, "channels [%d, %d) outside [0, %d)", cfg->chan0,
                    cfg->chan0 + cfg->n_chans, FE_H);
    if (!(cfg->gain > 0.f) || !(cfg->gain < 1e30f))
        return fail(XENG_EINVAL, "gain must be positive and finite");
    xeng_fengine *fe = new (std::nothrow) xeng_fengine;
    if (!fe) return fail(XENG_ENOMEM, "host allocation failed");
    fe->cfg = *cfg;
    // inputs per workgroup: the largest power of two up to 4 that divides them
    fe->group = 1;
    for (int g = FE_MAX_GROUP; g > 1; g >>= 1)
        if (cfg->n_inputs % g == 0) { fe->group = g; break; }

    // prototype: symmetric Hamming window times a sinc one channel wide,
    // coded as signed Q1.17 (18-bit) integers
    const int L = FE_TAPS * FE_P;
    const double pi = 3.14159265358979323846;
    std::vector<int32_t> coef(L);
    for (int l = 0; l < L; ++l) {
        const double w = 0.54 - 0.46 * std::cos(2.0 * pi * l / (L - 1));
        const double u = (l - (L - 1) / 2.0) / FE_P;
        const double s = u == 0.0 ? 1.0 : std::sin(pi * u) / (pi * u);
        const double c = std::nearbyint(w * s * 131072.0);
        coef[l] = (int32_t)std::min(131071.0, std::max(-131072.0, c));
    }
    std::vector<float2> tw(FE_TW_ROWS * 16), twr(FE_H);
    for (int row = 0; row < FE_TW_ROWS; ++row)
        for (int r = 0; r < 16; ++r) {
            const int k = row < 16 ? (row * r) % FE_H : ((row - 16) * r * 16) % FE_H;
            tw[row * 16 + r] = make_float2((float)std::cos(2.0 * pi * k / FE_H),
                                           (float)-std::sin(2.0 * pi * k / FE_H));
        }
    for (int k = 0; k < FE_H; ++k)
        twr[k] = make_float2((float)std::cos(2.0 * pi * k / FE_P), (float)-std::sin(2.0 * pi * k / FE_P));
    hipError_t e = hipMalloc((void **)&fe->d_coef, sizeof(int32_t) * L);
    if (e == hipSuccess) e = hipMalloc((void **)&fe->d_tw, sizeof(float2) * tw.size());
    if (e == hipSuccess) e = hipMalloc((void **)&fe->d_twr, sizeof(float2) * FE_H);
    if (e == hipSuccess) e = hipMemcpy(fe->d_coef, coef.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(fe->d_tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(fe->d_twr, twr.data(), sizeof(float2) * FE_H, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (fe->d_coef) (void)hipFree(fe->d_coef);
        if (fe->d_tw) (void)hipFree(fe->d_tw);
        if (fe->d_twr) (void)hipFree(fe->d_twr);
        delete fe;
        return fail(XENG_ENOMEM, "F-engine tables: %s", hipGetErrorString(e));
    }
    *out = fe;
    return XENG_OK;
}

int xeng_fengine_group(const xeng_fengine *fe)
{
    if (!fe) return fail(XENG_EINVAL, "fe is NULL");
    return fe->group;
}

int xeng_fengine_run(xeng_fengine *fe, const int8_t *d_adc, int64_t adc_stride, int64_t n_spectra,
                     uint8_t *d_out, void *d_spec, void *hip_stream)
{
    using namespace xeng;
    if (!fe || !d_adc || !d_out) return fail(XENG_EINVAL, "NULL argument");
    if (n_spectra < 1) return fail(XENG_EINVAL, "n_spectra %lld < 1", (long long)n_spectra);
    const int64_t need = (n_spectra + FE_TAPS - 1) * FE_P;
    if (adc_stride < need)
        return fail(XENG_EINVAL, "adc_stride %lld < %lld samples needed for %lld spectra",
                    (long long)adc_stride, (long long)need, (long long)n_spectra);
    if (((uintptr_t)d_adc & 7) || (adc_stride & 7))
        return fail(XENG_EINVAL, "ADC rows must start on 8-byte boundaries");
    const int G = fe->group;
    if ((uintptr_t)d_out % G || (d_spec && ((uintptr_t)d_spec & 7)))
        return fail(XENG_EINVAL, "output misaligned: out needs %d-byte, spec 8-byte alignment", G);
    const int n_groups = fe->cfg.n_inputs / G;
    const int64_t blocks = n_spectra * n_groups;
    if (blocks > 0x7FFFFFFF)
        return fail(XENG_EINVAL, "n_spectra x input groups %lld above one launch", (long long)blocks);
    FeArgs a;
    a.adc = d_adc;
    a.adc_stride = adc_stride;
    a.coef = fe->d_coef;
    a.tw = fe->d_tw;
    a.tw_r = fe->d_twr;
    a.out = d_out;
    a.spec = (float2 *)d_spec;
    a.n_inputs = fe->cfg.n_inputs;
    a.n_chans = fe->cfg.n_chans;
    a.chan0 = fe->cfg.chan0;
    a.group = G;
    a.n_groups = n_groups;
    a.n_blocks = (int32_t)blocks;
    a.scale = (float)((double)fe->cfg.gain / (131072.0 * FE_P));
    hipLaunchKernelGGL(fengine_kernel, dim3((unsigned)blocks), dim3(FE_THREADS), 0,
                       (hipStream_t)hip_stream, a);
    HIP_TRY(hipGetLastError());
    return XENG_OK;
}

int xeng_fengine_destroy(xeng_fengine *fe)
{
    if (!fe) return XENG_OK;
    (void)hipDeviceSynchronize();
    if (fe->d_coef) (void)hipFree(fe->d_coef);
    if (fe->d_tw) (void)hipFree(fe->d_tw);
    if (fe->d_twr) (void)hipFree(fe->d_twr);
    delete fe;
    return XENG_OK;
}

} // extern "C"
