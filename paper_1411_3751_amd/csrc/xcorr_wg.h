// Persistent-workgroup X-engine kernel (4-bit input with N a multiple of 16,
// 8-bit input with N a multiple of 8).
//
// Work is a host-built list of 128 x 128 tiles (subarray, channel, 128-input
// block I, block J <= I) of the lower block triangle of
// V[f] = sum_t x(t, f) x(t, f)^H (Section 2.5; Fig. 2 caption). Two
// workgroups of 4 waves run per CU; each walks its own slice of the list.
//
// Staging: each stage of a tile is copied raw ([time][128 I inputs | 128 J
// inputs], as stored in HBM) into a 4-deep LDS ring of 16 KB stages by
// buffer loads that write LDS directly, issued 3 stages ahead. A stage holds
// 64 time rows of 4-bit samples (256 bytes per row) or 32 rows of 8-bit
// samples (512 bytes). It is published to the four waves by one barrier
// after each wave's own copies have landed.
//
// Fragments: transposing LDS reads turn the time-major rows into the
// K-major operands of v_mfma_i32_32x32x32_i8 (lane l: input l % 32, K group
// l / 32). 4-bit rows use ds_read_b64_tr_b8: within each group of 16 lanes,
// lane 2m + h names time row m of half h of a 16-input chunk and lane 8h + j
// receives input 8h + j at 8 times. 8-bit rows use ds_read_b64_tr_b16 on
// (re, im) byte pairs: lane 4m + q names row m, quarter q of a 16-input span
// and lane k receives input k at 4 times; v_perm splits the pairs into re
// and im bytes.
//
// Each wave computes a 64 x 64 quarter of the tile as 2 x 2 MFMA tiles of
// 32 x 32. On a diagonal tile (J = I, only the I half is copied) the lower
// triangle is 10 such tiles. With 4-bit input on the int8 engine they are
// dealt as 20 half tiles (a half being one of the two K steps of every
// stage), 5 per wave: each wave multiplies two whole tiles and one half of
// a tile whose other half another wave multiplies, and the two halves are
// added through LDS at the flush. Otherwise waves 0, 1 take the diagonal
// quarters less their upper tile (3 each), waves 2, 3 the two 64 x 32
// columns below the first quarter (2 each).
//
// Operands: re, im and ~im (= -im - 1, so that -(-8) or -(-128) never has to
// fit in int8); 4-bit values are scaled by 16 by the nibble masks (see
// xcorr_i8.h). The int8 engines' imaginary sums are then Im V_ij - S_i with
// S_i = sum_t re_i. The accumulator keeps that raw form (the diagonal cell of
// row i then holds -S_i, since Im V_ii = 0, and the dump subtracts it); a
// sum that is exact already is a raw one with a zero diagonal, so both kinds
// of launch may add into one accumulator. A flush adds its sums to `src`
// (the accumulator, when it holds an earlier part of the integration) and
// writes `dst`. With FUSE (the last launch of a correlate-and-dump, dst the
// caller's output) each wave also sums S_i for its rows (v_dot8_i32_i4 on the
// raw 4-bit words with weight 1 on the real nibbles, v_dot4_i32_i8 on the
// 8-bit real parts) and the flush writes the exact V_ij: its own sums plus
// S_i, plus src minus src's diagonal word of row i.
#pragma once

#include <type_traits>

#include "xcorr_i8.h"

namespace xeng {

constexpr int WG_STAGE = 16384;                      // bytes per LDS stage
constexpr int WG_NBUF = 4;                           // LDS ring depth (stages)
constexpr int WG_DMA = WG_STAGE / (WG_THREADS * 16); // 16-byte copies per thread per stage (4)
constexpr int WG_MAX_SUBS = 16;

// Stage geometry per input width. A staged row is [128 I inputs | 128 J
// inputs] of one time sample; chunks are 16-byte copy units.
template <int IN_BITS> struct WgGeom;

template <> struct WgGeom<4> {
    static constexpr int TKS = 64;   // time rows per stage (two 32-sample K steps)
    static constexpr int ROWB = 256; // bytes per row
    static constexpr int NCH = 16;   // chunks per row
    static constexpr int CIN = 16;   // inputs per chunk
    static constexpr int BPS = 1;    // bytes per sample
    // chunk c of row tau sits in slot c ^ (tau & 7) ^ 8 (c & 1): the 8 rows a
    // tr8 group reads and the odd/even chunk pairs of neighbouring groups hit
    // distinct banks
    __device__ static int slot(int tau, int c) { return c ^ (tau & 7) ^ ((c & 1) << 3); }
    __device__ static int chunk(int tau, int sl)
    {
        const int c = sl ^ (tau & 7);
        return (c & 1) ? (c ^ 8) : c;
    }
};

template <> struct WgGeom<8> {
    static constexpr int TKS = 32;   // time rows per stage (one K step)
    static constexpr int ROWB = 512;
    static constexpr int NCH = 32;
    static constexpr int CIN = 8;
    static constexpr int BPS = 2;
    // chunk c of row tau sits in slot c ^ 4 (tau & 3): the 4 rows x 4 chunks
    // of one half-wave tr16 read cover 16 distinct 16-byte bank groups
    __device__ static int slot(int tau, int c) { return c ^ ((tau & 3) << 2); }
    __device__ static int chunk(int tau, int sl) { return sl ^ ((tau & 3) << 2); }
};

typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct WgSub {
    const uint8_t *samples; // [T][F][N] packed 4+4-bit
    const int32_t *src;     // sums to add ([F][tri(N)][2]), or null
    int32_t *dst;           // where the flush writes ([F][tri(N)][2])
    int64_t t_begin;        // first sample of this launch's segment
    int32_t t_count;        // samples in this segment (<= SEG_T), > 0
    int32_t n_chans;
    int32_t n_inputs;       // multiple of 16
    int32_t pad;
};

// Tile: chan | sub << 24, then bi | bj << 16 (128-input block indices).
struct WgItem {
    uint32_t cs;
    uint32_t ij;
};

struct WgArgs {
    WgSub subs[WG_MAX_SUBS];     // by value in the kernel arguments
    const WgItem *items;
    const int32_t *wg_begin;     // [n_wg + 1] item ranges per workgroup
};

// Wait until at most 4 * n of this wave's copies are outstanding and every
// LDS read it issued has returned, then barrier. The LDS wait keeps a slot's
// reads ahead of the copies into it: past the barrier another wave may copy
// a later stage into the slot a read of this wave came from, whether or not
// that read's data has been used yet.
__device__ __forceinline__ void wg_wait_barrier(int n)
{
    switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(16) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(20) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(24) lgkmcnt(0)\n\ts_barrier" ::: "memory"); break;
    }
}

// Raw fragments of one stage: [K step][side I/J][32-input block][load]
typedef i32x2 WgRaw[2][2][2][2];

// MFMA operands of one K step (32 samples)
struct WgOps {
    i32x4 reI[2], imI[2], reJ[2], imJ[2], niJ[2];
};

__device__ __forceinline__ u32x4 wg_raw(const WgRaw &R, int k, int sd, int blk)
{
    return u32x4{(uint32_t)R[k][sd][blk][0].x, (uint32_t)R[k][sd][blk][0].y,
                 (uint32_t)R[k][sd][blk][1].x, (uint32_t)R[k][sd][blk][1].y};
}

// ... and S[x] += the real parts of its I-side words (row sums for the Im
// correction): 4 v_dot8_i32_i4 with weights 1 on the real nibbles. IM, JM:
// the I and J blocks (bit x, bit y) that the K step's MFMAs use.
template <bool SUMS, int IM, int JM>
__device__ __forceinline__ void wg_unpack(const WgRaw &R, int k, WgOps &o, int32_t (&S)[2])
{
    static_assert(!SUMS || IM == 3, "row sums need every I block");
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        if (!((IM >> x) & 1)) continue;
        const u32x4 p = wg_raw(R, k, 0, x);
        o.reI[x] = (i32x4)(p & 0xF0F0F0F0u);
        o.imI[x] = (i32x4)((p << 4) & 0xF0F0F0F0u);
        if (SUMS) {
#pragma unroll
            for (int d = 0; d < 4; ++d) S[x] = __builtin_amdgcn_sdot8((int)p[d], 0x10101010, S[x], false);
        }
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        if (!((JM >> y) & 1)) continue;
        const u32x4 p = wg_raw(R, k, 1, y);
        const u32x4 im = (p << 4) & 0xF0F0F0F0u;
        o.reJ[y] = (i32x4)(p & 0xF0F0F0F0u);
        o.imJ[y] = (i32x4)im;
        o.niJ[y] = (i32x4)(im ^ 0xF0F0F0F0u);
    }
}

// 8-bit stage (one K step): raw load i (0..3) of (side, block) holds 4 times
// of (re, im) byte pairs; split them into re and im bytes.
__device__ __forceinline__ i32x2 wg8_raw(const WgRaw &R, int sd, int blk, int i)
{
    return R[i >> 1][sd][blk][i & 1];
}

__device__ __forceinline__ void wg8_split(const WgRaw &R, int sd, int blk, i32x4 &re, i32x4 &im)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const i32x2 v = wg8_raw(R, sd, blk, i);
        re[i] = (int32_t)__builtin_amdgcn_perm((uint32_t)v.y, (uint32_t)v.x, 0x06040200u);
        im[i] = (int32_t)__builtin_amdgcn_perm((uint32_t)v.y, (uint32_t)v.x, 0x07050301u);
    }
}

template <bool SUMS, int NY>
__device__ __forceinline__ void wg8_unpack(const WgRaw &R, WgOps &o, int32_t (&S)[2])
{
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        wg8_split(R, 0, x, o.reI[x], o.imI[x]);
        if (SUMS) {
#pragma unroll
            for (int d = 0; d < 4; ++d)
                S[x] = __builtin_amdgcn_sdot4(o.reI[x][d], 0x01010101, S[x], false);
        }
    }
#pragma unroll
    for (int y = 0; y < NY; ++y) {
        wg8_split(R, 1, y, o.reJ[y], o.imJ[y]);
        o.niJ[y] = ~o.imJ[y];
    }
}

// The MFMAs of blocks [b0, b1) of one K step that MASK names (bit b), blocks
// in the order b = (x, y) = (0, 0), (1, 0), (0, 1), (1, 1):
//   accR[x][y] += re_I re_J + im_I im_J,  accI[x][y] += re_I ~im_J + im_I re_J.
template <int B0, int B1, int MASK>
__device__ __forceinline__ void wg_mfma_blocks(const WgOps &o, i32x16 (&accR)[2][2],
                                               i32x16 (&accI)[2][2])
{
#pragma unroll
    for (int b = B0; b < B1; ++b) {
        if (!((MASK >> b) & 1)) continue;
        const int x = b & 1, y = b >> 1;
        accR[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.reI[x], o.reJ[y], accR[x][y], 0, 0, 0);
        accI[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.reI[x], o.niJ[y], accI[x][y], 0, 0, 0);
        accR[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.imI[x], o.imJ[y], accR[x][y], 0, 0, 0);
        accI[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.imI[x], o.reJ[y], accI[x][y], 0, 0, 0);
    }
}

// Blocks of the last K step issued before the next stage is published and
// its fragments are read (the rest are issued after, covering the reads'
// latency; the ones before cover the barrier's wait). Measured best: half
// for 4-bit input (two K steps per stage), one block for 8-bit (one K step).
template <int IN_BITS> constexpr int wg_split() { return IN_BITS == 4 ? 2 : 1; }

// The I blocks (bit x) and J blocks (bit y) that the blocks of MASK use.
constexpr int wg_imask(int m) { return ((m & 5) ? 1 : 0) | ((m & 10) ? 2 : 0); }
constexpr int wg_jmask(int m) { return ((m & 3) ? 1 : 0) | ((m & 12) ? 2 : 0); }

// The v_mfma_i32_32x32x32_i8 of one K step over the 2 x 2 tiles of 32 x 32
// that MASK names:
//   accR[x][y] += re_I re_J + im_I im_J,  accI[x][y] += re_I ~im_J + im_I re_J.
template <int MASK>
__device__ __forceinline__ void wg_mfma(const WgOps &o, i32x16 (&accR)[2][2], i32x16 (&accI)[2][2])
{
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            if (!((MASK >> (x + 2 * y)) & 1)) continue;
            accR[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.reI[x], o.reJ[y], accR[x][y], 0, 0, 0);
            accI[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.reI[x], o.niJ[y], accI[x][y], 0, 0, 0);
            accR[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.imI[x], o.imJ[y], accR[x][y], 0, 0, 0);
            accI[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.imI[x], o.reJ[y], accI[x][y], 0, 0, 0);
        }
}

// ---- FP8 engine (OCP e4m3 operands, fp32 accumulation) -----------------
//
// Operands are offset values u = v + 8 in 0..15 (the nibble with its sign
// bit flipped: two bit operations per 4 samples). The e4m3 code whose bit
// pattern is u stands for u * 2^-9 exactly (0..7 are the subnormals m * 2^-9,
// 8..15 the first normal binade (1 + m/8) * 2^-6), so with block scales of
// 2^9 on both operands every product is the exact integer u_a u_b; the sign
// bit negates a code exactly. Per K step and 32 x 32 block:
//   accR += u(re_I) u(re_J) + u(im_I) u(im_J),
//   accI += u(im_I) u(re_J) - u(re_I) u(im_J),
// so that, with P_n = sum_t u(re_n), Q_n = sum_t u(im_n) over the launch's
// rows (T' of them, the zero rows that pad a segment to whole stages
// included: for them every u is 8 and every difference below is 0),
//   Re V_ij = accR - 8 (P_i + Q_i + P_j + Q_j) + 128 T',
//   Im V_ij = accI - 8 (Q_i - P_i) + 8 (Q_j - P_j).
// Each wave sums P and Q of its own I rows and J columns (byte-wise adds of
// the 8 code words of a fragment, at most 8 * 15 per byte, then one
// v_sad_u8); the flush applies the correction, so the accumulator holds the
// exact sums, as the raw convention allows. The fp32 sums stay exact: a
// segment of at most SEG_T = 2^15 samples keeps |accR| <= 2^15 * 450 < 2^24.
constexpr int ENG_I8 = 0;
constexpr int ENG_F8 = 1;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));

constexpr int F8_SCALE = 127 + 9; // E8M0 block scale 2^9 on each operand

// offset codes of the real parts (high nibbles) of 4 packed samples
__device__ __forceinline__ uint32_t f8_re(uint32_t w) { return ((w >> 4) & 0x0F0F0F0Fu) ^ 0x08080808u; }

// offset codes of the imaginary parts (low nibbles) of 4 packed samples
__device__ __forceinline__ uint32_t f8_im(uint32_t w) { return (w & 0x0F0F0F0Fu) ^ 0x08080808u; }

// raw dword d (0..7) of side sd, block blk of a stage: K steps 0 and 1 of
// the int8 layout concatenated (A and B lanes hold the same samples at the
// same positions, so any fixed order of K within the lane is valid)
__device__ __forceinline__ uint32_t wg_raw_dw(const WgRaw &R, int sd, int blk, int d)
{
    const i32x2 v = R[d >> 2][sd][blk][(d >> 1) & 1];
    return (uint32_t)((d & 1) ? v.y : v.x);
}

// this lane's part of the sum of the 32 codes of a fragment (8 words)
__device__ __forceinline__ int32_t f8_sum(const i32x8 &c, int32_t acc)
{
    const uint32_t b = (uint32_t)c[0] + (uint32_t)c[1] + (uint32_t)c[2] + (uint32_t)c[3] + (uint32_t)c[4] +
                       (uint32_t)c[5] + (uint32_t)c[6] + (uint32_t)c[7];
    return (int32_t)__builtin_amdgcn_sad_u8(b, 0u, (uint32_t)acc);
}

// Code sums of the two fragments a wave sums: P (real) and Q (imaginary) of
// I block sx (a) and J block sy (b), this lane's half of row / column l % 32.
// Each input of a tile is summed by one wave only, and the flush shares the
// sums through LDS.
struct F8Sums {
    int32_t pa, qa, pb, qb;
};

// One stage (64 samples) of the FP8 engine on the 2 x 2 tiles of 32 x 32
// that both MASK and the wave-uniform rmask name (a J fragment no tile uses
// is not converted): v_mfma_scale_f32_32x32x64_f8f6f4 with scales 2^9, and
// the code sums of the fragments sx, sy.
template <int MASK>
__device__ __forceinline__ void wg_f8_stage(const WgRaw &R, f32x16 (&accR)[2][2], f32x16 (&accI)[2][2],
                                            F8Sums &sm, int sx, int sy, int rmask)
{
    i32x8 reI[2], imI[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const uint32_t w = wg_raw_dw(R, 0, x, d);
            reI[x][d] = (int32_t)f8_re(w);
            imI[x][d] = (int32_t)f8_im(w);
        }
        if (sx == x) {
            sm.pa = f8_sum(reI[x], sm.pa);
            sm.qa = f8_sum(imI[x], sm.qa);
        }
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        if (!((MASK >> (2 * y)) & 3) || !((rmask >> (2 * y)) & 3)) continue; // no block of this J column
        // the negated imaginary operand replaces the plain one in the same
        // registers once the plain one's products are issued
        i32x8 reJ, imJ;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const uint32_t w = wg_raw_dw(R, 1, y, d);
            reJ[d] = (int32_t)f8_re(w);
            imJ[d] = (int32_t)f8_im(w);
        }
        if (sy == y) {
            sm.pb = f8_sum(reJ, sm.pb);
            sm.qb = f8_sum(imJ, sm.qb);
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            if (!((MASK >> (x + 2 * y)) & 1) || !((rmask >> (x + 2 * y)) & 1)) continue;
            accR[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(reI[x], reJ, accR[x][y], 0, 0, 0,
                                                                         F8_SCALE, 0, F8_SCALE);
            accI[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(imI[x], reJ, accI[x][y], 0, 0, 0,
                                                                         F8_SCALE, 0, F8_SCALE);
            accR[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(imI[x], imJ, accR[x][y], 0, 0, 0,
                                                                         F8_SCALE, 0, F8_SCALE);
        }
        const i32x8 niJ = imJ ^ (int32_t)0x80808080u;
#pragma unroll
        for (int x = 0; x < 2; ++x)
            if (((MASK >> (x + 2 * y)) & 1) && ((rmask >> (x + 2 * y)) & 1))
                accI[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(reI[x], niJ, accI[x][y], 0, 0,
                                                                             0, F8_SCALE, 0, F8_SCALE);
    }
}

// accumulator element -> int32 word of the raw accumulator (4-bit int8
// products carry a factor 256)
template <int IN_BITS>
__device__ __forceinline__ uint32_t acc_word(int32_t v) { return (uint32_t)(IN_BITS == 4 ? v >> 8 : v); }
template <int IN_BITS>
__device__ __forceinline__ uint32_t acc_word(float v) { return (uint32_t)(int32_t)v; }

// Two workgroups per CU (launch bounds 256 threads x 2): each one's barrier
// and LDS latency is covered by the other's MFMAs.
template <int ENG, int IN_BITS, bool FUSE>
__global__ __launch_bounds__(WG_THREADS, 2) void xcorr_wg_kernel(WgArgs a)
{
    static_assert(ENG == ENG_I8 || IN_BITS == 4, "the FP8 engine takes 4-bit input");
    typedef WgGeom<IN_BITS> Geo;
    static_assert(Geo::TKS * Geo::ROWB == WG_STAGE, "stage size");
    typedef typename std::conditional<ENG == ENG_F8, f32x16, i32x16>::type AccT;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WG_NBUF * WG_STAGE];
    // Diagonal tiles split by K step (4-bit input on the int8 engine)
    constexpr bool KSPLIT = ENG == ENG_I8 && IN_BITS == 4;
    // FP8 engine: code sums of a tile's inputs by staged-row position, P then
    // Q. K-split diagonal tiles: -S_i of the tile's rows i, for the waves
    // whose blocks hold no diagonal cell of those rows.
    __shared__ int32_t f8t[ENG == ENG_F8 ? 2 * 256 : (KSPLIT ? 128 : 1)];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wave-uniform values go through readfirstlane so that the item and
    // descriptor loads are scalar loads (a vector load would make the
    // compiler wait for all vector memory traffic, draining the copy ring)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    typedef __attribute__((address_space(4))) const uint32_t c_u32_t;
    typedef __attribute__((address_space(4))) const int32_t c_i32_t;
    c_u32_t *itw = (c_u32_t *)a.items;
    c_i32_t *wbeg = (c_i32_t *)a.wg_begin;
    const int it_begin = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x]);
    const int it_end = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x + 1]);
    if (it_begin >= it_end) return; // the same for every wave of the workgroup
    auto item_at = [&](int it) {
        const int u = __builtin_amdgcn_readfirstlane(it);
        WgItem w;
        w.cs = itw[2 * u];
        w.ij = itw[2 * u + 1];
        return w;
    };
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    constexpr uint32_t OOR = 0x80000000u;
    constexpr int TKS = Geo::TKS;

    // ---- copy cursor (every thread follows the same sequence of stages)
    int d_item = it_begin, d_stage = 0, d_nstage = 0, d_tcount = 0;
    const uint8_t *d_base = nullptr;
    uint32_t d_rowstride = 0;
    uint32_t d_voff[WG_DMA];
    auto d_setup = [&](int it) {
        const WgItem w = item_at(it);
        const WgSub &sb = a.subs[w.cs >> 24];
        const int f = (int)(w.cs & 0xFFFFFFu);
        const int bi = (int)(w.ij & 0xFFFFu), bj = (int)(w.ij >> 16);
        const int N = sb.n_inputs;
        d_rowstride = (uint32_t)sb.n_chans * (uint32_t)N * Geo::BPS;
        d_tcount = sb.t_count;
        d_nstage = (sb.t_count + TKS - 1) / TKS;
        d_base = sb.samples + ((size_t)sb.t_begin * sb.n_chans + f) * (size_t)N * Geo::BPS;
        const bool diag = bi == bj;
#pragma unroll
        for (int k = 0; k < WG_DMA; ++k) {
            const int P = k * WG_THREADS + tid;  // 16-byte position in the stage
            const int tau = P / Geo::NCH, sl = P % Geo::NCH;
            const int c = Geo::chunk(tau, sl);
            const int hc = Geo::NCH / 2;
            const int in = c < hc ? 128 * bi + Geo::CIN * c : 128 * bj + Geo::CIN * (c - hc);
            // a diagonal tile reads its J operands from the I half
            const bool on = in < N && !(diag && c >= hc);
            d_voff[k] = on ? (uint32_t)tau * d_rowstride + (uint32_t)(in * Geo::BPS) : OOR;
        }
    };
    int issued = 0;
    auto d_issue = [&]() {
        const int t_first = d_stage * TKS;
        const int nt = d_tcount - t_first < TKS ? d_tcount - t_first : TKS;
        const uint64_t base = (uint64_t)(uintptr_t)(d_base + (size_t)t_first * d_rowstride);
        const i32x4 rsrc = {(int)(uint32_t)base, (int)((uint32_t)(base >> 32) & 0xFFFFu),
                            (int)((uint32_t)nt * d_rowstride), 0x00020000};
        const uint32_t dst = lds_base + (uint32_t)((issued % WG_NBUF) * WG_STAGE + wave * 1024);
#pragma unroll
        for (int k = 0; k < WG_DMA; ++k)
            dma16(rsrc, d_voff[k], dst + (uint32_t)(k * WG_THREADS * 16));
        ++issued;
        if (++d_stage == d_nstage) {
            d_stage = 0;
            if (++d_item < it_end) d_setup(d_item);
        }
    };

    int n_total = 0;
    for (int it = it_begin; it < it_end; ++it) {
        const WgSub &sb = a.subs[item_at(it).cs >> 24];
        n_total += (sb.t_count + TKS - 1) / TKS;
    }
    d_setup(it_begin);
#pragma unroll
    for (int k = 0; k < WG_NBUF - 1; ++k)
        if (issued < n_total) d_issue();

    // This wave's part of a tile: its 32-input I blocks x = 0, 1 start at
    // staged-row positions ipos[x] (tile rows ipos[x]), its J blocks y at
    // jpos[y] (the J half starts at 128; tile columns jpos[y] - 128, or
    // jpos[y] on a diagonal tile, where J = I and only the I half is
    // copied). Its MFMA blocks are (x, y), bit x + 2 y of a mask.
    //   kind 0, off the diagonal: a 64 x 64 quarter (4 blocks).
    // A diagonal tile has 10 lower-triangle blocks of 32 x 32 (tile blocks
    // (a, b), b <= a).
    //   kinds 1, 2 (FP8 engine, 8-bit input): waves 0, 1 take the diagonal
    //   quarters without their upper block (3 blocks each), waves 2, 3 the
    //   blocks of rows 64..127 in columns 0..31 and 32..63 (2 blocks each).
    //   kinds 3, 4 (4-bit input on the int8 engine): 5 half blocks each, a
    //   half block being one of the two K steps of every stage. Tile blocks
    //   (0, 0) and (2, 1) are split: waves 0, 1 (kind 3) multiply their half
    //   (accumulator slot (x, y) = (1, 1)) in the first K step of every
    //   stage, waves 2, 3 (kind 4) theirs (slot (0, 0)) in the second; the
    //   halves meet at the flush.
    //     wave 0: I blocks (1, 2), J blocks (0, 1): (1,0) (1,1), half (2,1)
    //     wave 1: I blocks (2, 0), J blocks (2, 0): (2,2) (2,0), half (0,0)
    //     wave 2: I blocks (0, 3), J blocks (0, 2): (3,0) (3,2), half (0,0)
    //     wave 3: I blocks (2, 3), J blocks (1, 3): (3,1) (3,3), half (2,1)
    struct Role {
        int ipos[2], jpos[2], kind;
    };
    auto role = [&](const WgItem &w) {
        const int bi = (int)(w.ij & 0xFFFFu), bj = (int)(w.ij >> 16);
        Role r;
        if (bi != bj) {
            const int wr = wave >> 1, wc = wave & 1;
            r.ipos[0] = 64 * wr;
            r.jpos[0] = 128 + 64 * wc;
            r.ipos[1] = r.ipos[0] + 32;
            r.jpos[1] = r.jpos[0] + 32;
            r.kind = 0;
        } else if constexpr (KSPLIT) {
            // tile blocks of the table above, one nibble per wave
            r.ipos[0] = 32 * ((0x2021 >> (4 * wave)) & 3);
            r.ipos[1] = 32 * ((0x3302 >> (4 * wave)) & 3);
            r.jpos[0] = 32 * ((0x1020 >> (4 * wave)) & 3);
            r.jpos[1] = 32 * ((0x3201 >> (4 * wave)) & 3);
            r.kind = wave < 2 ? 3 : 4;
        } else if (wave < 2) {
            r.ipos[0] = r.jpos[0] = 64 * wave;
            r.ipos[1] = r.jpos[1] = 64 * wave + 32;
            r.kind = 1;
        } else {
            r.ipos[0] = 64;
            r.ipos[1] = 96;
            r.jpos[0] = 32 * (wave - 2);
            r.jpos[1] = r.jpos[0] + 32;
            r.kind = 2;
        }
        return r;
    };

    // ---- read cursor: the stage whose fragments are read next, and the
    // transposing-load offsets of its tile's role. The rows of the loads of
    // one (side, block) differ by multiples of 8 (4-bit) or 4 (8-bit) from
    // the lane's base row, so they share its slot swizzle: one register per
    // (side, block), the rest are immediate offsets.
    const int G = lane >> 4;
    int fo[2][2]; // (side, block) -> byte offset of load 0 in a stage
    int r_item = it_begin, r_stage = 0, r_nstage = 0, r_tcount = 0;
    auto r_setup = [&](int it) {
        const WgItem w = item_at(it);
        const WgSub &sb = a.subs[w.cs >> 24];
        r_tcount = sb.t_count;
        r_nstage = (sb.t_count + TKS - 1) / TKS;
        const Role ro = role(w);
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                const int pos = (sd == 0 ? ro.ipos[blk] : ro.jpos[blk]) + 16 * (G & 1);
                if constexpr (IN_BITS == 4) {
                    const int m = (lane >> 1) & 7, h = lane & 1;
                    const int tau = 16 * (G >> 1) + m;
                    const int c = pos / Geo::CIN;
                    fo[sd][blk] = tau * Geo::ROWB + 16 * Geo::slot(tau, c) + 8 * h;
                } else {
                    const int m = (lane >> 2) & 3, q = lane & 3;
                    const int tau = 16 * (G >> 1) + m;
                    const int c = pos / Geo::CIN + (q >> 1);
                    fo[sd][blk] = tau * Geo::ROWB + 16 * Geo::slot(tau, c) + 8 * (q & 1);
                }
            }
    };

    // Make the read cursor's stage s visible to every wave: this wave's
    // copies of it are done once at most the later issued stages are
    // outstanding; then barrier. Rows past the end of the segment are
    // cleared cooperatively.
    auto prep_stage = [&](int s) {
        const int later = issued - (s + 1);
        if (later >= WG_NBUF - 2) wg_wait_barrier(WG_NBUF - 2);
        else if (later >= 1) wg_wait_barrier(1);
        else wg_wait_barrier(0);
        const int nt = r_tcount - r_stage * TKS;
        if (nt < TKS) {
            uint8_t *b = lds + (s % WG_NBUF) * WG_STAGE;
            for (int o = tid * 16; o < WG_STAGE; o += WG_THREADS * 16)
                if (o / Geo::ROWB >= nt) *(u32x4 *)(b + o) = u32x4{0u, 0u, 0u, 0u};
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
    };
    auto r_advance = [&]() {
        if (++r_stage == r_nstage) {
            r_stage = 0;
            if (++r_item < it_end) r_setup(r_item);
        }
    };
    // K steps [K0, K1) of a stage's fragments into R, at the offsets fo
    // (the read cursor's stage) or, for the second K step of the stage being
    // multiplied, fo_mul: the offsets of that stage's role, kept when its
    // first K step was read (the cursor has moved on, possibly to a tile of
    // another role)
    int fo_mul[2][2];
    auto read_frags_k = [&](int slot, WgRaw &R, auto k0_c, auto k1_c) {
        constexpr int K0 = decltype(k0_c)::value, K1 = decltype(k1_c)::value;
        const uint8_t *b = lds + slot * WG_STAGE;
        if constexpr (K0 == 0) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd)
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) fo_mul[sd][blk] = fo[sd][blk];
        }
#pragma unroll
        for (int k = K0; k < K1; ++k)
#pragma unroll
            for (int sd = 0; sd < 2; ++sd)
#pragma unroll
                for (int blk = 0; blk < 2; ++blk)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        if constexpr (IN_BITS == 4) {
                            // K step k, rows 8 i apart
                            R[k][sd][blk][i] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                                (lds_i32x2 *)(b + fo_mul[sd][blk] + (32 * k + 8 * i) * Geo::ROWB));
                        } else {
                            // load 2 k + i, rows 4 (2 k + i) apart
                            R[k][sd][blk][i] = (i32x2)__builtin_amdgcn_ds_read_tr16_b64_v4i16(
                                (lds_i16x4 *)(b + fo_mul[sd][blk] + 4 * (2 * k + i) * Geo::ROWB));
                        }
                    }
    };
    auto read_frags = [&](int slot, WgRaw &R) {
        read_frags_k(slot, R, std::integral_constant<int, 0>{}, std::integral_constant<int, 2>{});
    };
    // 4-bit input on the int8 engine reads a stage's second K step only when
    // the stage is multiplied (the first right after the barrier that
    // publishes it): two bursts of 8 reads instead of one of 16, the second
    // covered by the first K step's MFMAs
    constexpr bool SPLIT_READS = ENG == ENG_I8 && IN_BITS == 4;

    AccT accR[2][2], accI[2][2];
    WgRaw RA;
    WgOps O0;
    r_setup(it_begin);
    prep_stage(0);
    if constexpr (SPLIT_READS)
        read_frags_k(0, RA, std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    else
        read_frags(0, RA);
    r_advance();
    int s = 0; // global index of the stage being multiplied

    for (int it = it_begin; it < it_end; ++it) {
        const WgItem w = item_at(it);
        const WgSub &sb = a.subs[w.cs >> 24];
        const int f = (int)(w.cs & 0xFFFFFFu);
        const int nst = (sb.t_count + TKS - 1) / TKS;
        const Role ro = role(w);
        const int kind = ro.kind;
        const int ip = ro.ipos[0], jp = ro.jpos[0]; // first blocks (kinds 0..2: the second is 32 on)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                accR[x][y] = AccT{};
                accI[x][y] = AccT{};
            }
        int32_t S[2] = {0, 0}; // this lane's part of S_i of rows l % 32 of I blocks 0, 1 (FUSE)
        F8Sums sm = {};        // FP8 engine: code sums of the fragments
        // which fragments this wave sums: off the diagonal I block (wave & 1)
        // and J block (wave >> 1); on it (J = I) waves 0 and 1 sum inputs
        // 0..63 and 64..127 (their I block 0 and J block 1), waves 2, 3 none
        // FP8 engine: the blocks of the role (kinds 0..2), skipped by
        // wave-uniform branches in the one stage loop
        const int f8_mask =
            ENG == ENG_F8 ? __builtin_amdgcn_readfirstlane(kind == 1 ? 0xB : kind == 2 ? 0x3 : 0xF) : 0xF;
        const int sx = kind == 0 ? (wave & 1) : (wave < 2 ? 0 : -1);
        const int sy = kind == 0 ? (wave >> 1) : (wave < 2 ? 1 : -1);
        // The stage loop of one role kind (M0, M1: its blocks in the first and
        // the second K step of a stage; one K step for 8-bit input, M0 = M1).
        // The stage's fragments were read by the previous step (RA). Once its
        // last K step is unpacked RA is free, so the next stage is published
        // and read into RA between the first wg_split() blocks of that K
        // step's MFMAs and the rest: the MFMAs before the barrier cover its
        // wait, those after cover the reads' latency. SUMS_C: the role sums
        // S_i of its rows (the other roles find them on a diagonal cell).
        auto stages = [&](auto m0_c, auto m1_c, auto sums_c) {
            constexpr int M0 = decltype(m0_c)::value, M1 = decltype(m1_c)::value;
            constexpr bool SUMS = FUSE && decltype(sums_c)::value;
            static_assert(IN_BITS == 4 || M0 == M1, "one K step per stage");
            for (int k = 0; k < nst; ++k, ++s) {
                if (issued < n_total) d_issue();
                const bool more = s + 1 < n_total;
                if constexpr (ENG == ENG_F8) {
                    wg_f8_stage<M0>(RA, accR, accI, sm, sx, sy, f8_mask);
                    // the next stage's reads stay behind this stage's MFMAs
                    // (hoisted above them they would hold RA live beside the
                    // codes)
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) {
                        prep_stage(s + 1);
                        read_frags((s + 1) % WG_NBUF, RA);
                    }
                } else {
                    if constexpr (SPLIT_READS)
                        read_frags_k(s % WG_NBUF, RA, std::integral_constant<int, 1>{},
                                     std::integral_constant<int, 2>{});
                    if constexpr (IN_BITS == 4) {
                        wg_unpack<SUMS, wg_imask(M0), wg_jmask(M0)>(RA, 0, O0, S);
                        wg_mfma<M0>(O0, accR, accI);
                        wg_unpack<SUMS, wg_imask(M1), wg_jmask(M1)>(RA, 1, O0, S);
                    } else {
                        wg8_unpack<SUMS, (M1 & 0xC) ? 2 : 1>(RA, O0, S);
                    }
                    wg_mfma_blocks<0, wg_split<IN_BITS>(), M1>(O0, accR, accI);
                    // Every fragment read of this stage has returned by now
                    // (the barrier below waits for them anyway). A wait the
                    // compiler sees keeps it from making the blocks after the
                    // barrier wait for the next stage's reads where the paths
                    // with and without them join.
                    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0)
                    if (more) {
                        prep_stage(s + 1);
                        if constexpr (SPLIT_READS)
                            read_frags_k((s + 1) % WG_NBUF, RA, std::integral_constant<int, 0>{},
                                         std::integral_constant<int, 1>{});
                        else
                            read_frags((s + 1) % WG_NBUF, RA);
                    }
                    wg_mfma_blocks<wg_split<IN_BITS>(), 4, M1>(O0, accR, accI);
                }
                if (more) r_advance();
            }
        };
        using std::integral_constant;
        using std::bool_constant;
        if constexpr (ENG == ENG_F8) {
            // one stage loop for every role, the role's blocks chosen at run
            // time (f8_mask): a single copy of the FP8 loop leaves its
            // register allocation room
            stages(integral_constant<int, 0xF>{}, integral_constant<int, 0xF>{}, bool_constant<false>{});
        } else if (kind == 0) {
            stages(integral_constant<int, 0xF>{}, integral_constant<int, 0xF>{}, bool_constant<true>{});
        } else if constexpr (KSPLIT) {
            // split block in slot (1, 1), first K step / in slot (0, 0), second K step
            if (kind == 3)
                stages(integral_constant<int, 0xD>{}, integral_constant<int, 0x5>{}, bool_constant<false>{});
            else
                stages(integral_constant<int, 0xA>{}, integral_constant<int, 0xB>{}, bool_constant<false>{});
        } else if (kind == 1) {
            stages(integral_constant<int, 0xB>{}, integral_constant<int, 0xB>{}, bool_constant<false>{});
        } else {
            stages(integral_constant<int, 0x3>{}, integral_constant<int, 0x3>{}, bool_constant<true>{});
        }

        // ---- flush. 32 x 32 MFMA result: lane l holds column l % 32 of rows
        // 8 (r / 4) + 4 (l / 32) + r % 4. Buffer loads / stores relative to
        // the tile's first row: elements above the diagonal, past N, or in a
        // block the wave does not own get an out-of-range offset (loads read
        // 0, stores are dropped), no branches. S: lanes l and l + 32 hold
        // halves of the row sum of row l % 32 of I block x; the int8 engines
        // add it to Im. Roles without sums take S_i from a diagonal cell
        // (Im V_ii = 0, so the raw diagonal word is -S_i): their own, or one
        // another wave left in f8t.
        const int N = sb.n_inputs;
        const int bi = (int)(w.ij & 0xFFFFu), bj = (int)(w.ij >> 16);
        const int I0 = 128 * bi, J0 = 128 * bj;
        const int cofs = bi == bj ? 0 : 128; // J positions -> tile columns
        // blocks (bit x + 2 y) this wave writes
        const int own = kind == 2 ? 0x3 : kind == 3 ? 0xD : kind == 4 ? 0xA : 0xF;
        // per I block x, where S_i comes from: -1 the wave's sums (or no
        // rows), 0 / 1 the diagonal cell of its block (x, 0) / (x, 1), 2 f8t
        const int sdy0 = kind == 1 ? 0 : kind == 3 ? (wave == 0 ? 1 : 0) : -1;
        const int sdy1 = kind == 1 ? 1 : kind == 3 ? (wave == 0 ? 2 : 1) : kind == 4 ? (wave == 2 ? 2 : 1) : -1;
        // lane-derived flush offsets from an opaque copy of the lane index, so
        // that they are not hoisted out of the tile loop (and kept live in
        // registers across the stage loop)
        int fl = lane;
        asm volatile("" : "+v"(fl));
        const int lh = fl >> 5, lc = fl & 31;
        // the accumulator word of diagonal cell (lc, lc) of a block, in the
        // lane that holds it (lane half (lc / 4) % 2, register
        // 4 (lc / 8) + lc % 4), 0 in the other lane of the pair
        auto diag_word = [&](const AccT &v) {
            const int ri = 4 * (lc >> 3) + (lc & 3);
            int32_t d = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) d = r == ri ? (int32_t)acc_word<IN_BITS>(v[r]) : d;
            return ((lc >> 2) & 1) == lh ? d : 0;
        };
        if constexpr (KSPLIT) {
            if (kind >= 3) {
                // Split blocks: waves 2, 3 hand their half of slot (0, 0) to
                // waves 1, 0 (slot (1, 1)) through the LDS stage of the
                // tile's last stage (every wave is done with it; its next
                // copy is issued after the flush), 8 KB each. Waves 1 and 3
                // leave -S_i of tile rows 64..127 (their diagonal cells of
                // tile blocks (2, 2) and (3, 3)) in f8t.
                uint8_t *mb = lds + ((s - 1) % WG_NBUF) * WG_STAGE;
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                if (kind == 4) {
                    u32x4 *dst = (u32x4 *)(mb + (3 - wave) * 8192) + lane;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        dst[64 * c] = u32x4{(uint32_t)accR[0][0][4 * c], (uint32_t)accR[0][0][4 * c + 1],
                                            (uint32_t)accR[0][0][4 * c + 2], (uint32_t)accR[0][0][4 * c + 3]};
                        dst[64 * (4 + c)] = u32x4{(uint32_t)accI[0][0][4 * c], (uint32_t)accI[0][0][4 * c + 1],
                                                  (uint32_t)accI[0][0][4 * c + 2], (uint32_t)accI[0][0][4 * c + 3]};
                    }
                }
                if (FUSE && (wave & 1)) {
                    const int x = wave == 1 ? 0 : 1;
                    const int32_t dv = diag_word(wave == 1 ? accI[0][0] : accI[1][1]);
                    if (((lc >> 2) & 1) == lh) f8t[ro.ipos[x] + lc] = dv;
                }
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                if (kind == 3) {
                    const u32x4 *src = (const u32x4 *)(mb + wave * 8192) + lane;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const u32x4 pr = src[64 * c], pi = src[64 * (4 + c)];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            accR[1][1][4 * c + e] += (int32_t)pr[e];
                            accI[1][1][4 * c + e] += (int32_t)pi[e];
                        }
                    }
                }
            }
        }
        const int64_t tri = (int64_t)N * (N + 1) / 2;
        const int r1 = I0 + 128 < N ? I0 + 128 : N;
        const int64_t rb0 = (int64_t)I0 * (I0 + 1) / 2;
        const int64_t rb1 = (int64_t)r1 * (r1 + 1) / 2;
        const size_t cell0 = (size_t)f * (size_t)tri + (size_t)rb0;
        const int nbytes = (int)((rb1 - rb0) * 8);
        const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((uint2 *)sb.dst + cell0), (short)0, nbytes, 0x00020000);
        const bool add = sb.src != nullptr;
        const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const uint2 *)(add ? sb.src : sb.dst) + cell0), (short)0, add ? nbytes : 0,
            0x00020000);
        if constexpr (FUSE) {
            // S[x] of row l % 32 of I block x: this wave's sums (int8 engines)
            // minus src's diagonal word of that row (src's own -S_i, or 0)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                if (ENG == ENG_I8) S[x] += __shfl_xor(S[x], 32);
                const int i = I0 + ro.ipos[x] + lc;
                const uint32_t doff = (i < N) ? (uint32_t)((int64_t)i * (i + 1) / 2 + i - rb0) * 8u : OOR;
                const u32x2 dg = add ? __builtin_amdgcn_raw_buffer_load_b64(srs, (int)doff, 0, 0)
                                     : u32x2{0u, 0u};
                S[x] -= (int32_t)dg.y;
                if constexpr (ENG == ENG_I8) {
                    const int sdy = x == 0 ? sdy0 : sdy1;
                    if (sdy == 0 || sdy == 1) {
                        const int32_t dv = diag_word(sdy == 0 ? accI[x][0] : accI[x][1]);
                        S[x] -= dv + __shfl_xor(dv, 32);
                    } else if (KSPLIT && sdy == 2) {
                        S[x] -= f8t[ro.ipos[x] + lc];
                    }
                }
            }
        }
        if constexpr (KSPLIT) {
            // the merge area is free again once every wave has read it
            if (kind >= 3) asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
        // FP8 engine: the offset correction, per row (lanes l and l + 32 hold
        // halves of row l % 32's sums; the row's value is fetched by its
        // lanes) and per column (this lane's own column l % 32)
        int32_t fr[2] = {0, 0}, fi[2] = {0, 0}, gr[2] = {0, 0}, gi[2] = {0, 0};
        if constexpr (ENG == ENG_F8) {
            // this wave's sums into the table (full sums: both halves), then
            // every wave's rows and columns out of it
            const int32_t pa = sm.pa + __shfl_xor(sm.pa, 32), qa = sm.qa + __shfl_xor(sm.qa, 32);
            const int32_t pb = sm.pb + __shfl_xor(sm.pb, 32), qb = sm.qb + __shfl_xor(sm.qb, 32);
            // (every wave is done reading the previous tile's table)
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            if (lh == 0 && sx >= 0) {
                f8t[ip + 32 * sx + lc] = pa;
                f8t[256 + ip + 32 * sx + lc] = qa;
            }
            if (lh == 0 && sy >= 0) {
                f8t[jp + 32 * sy + lc] = pb;
                f8t[256 + jp + 32 * sy + lc] = qb;
            }
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int32_t p = f8t[ip + 32 * x + lc], q = f8t[256 + ip + 32 * x + lc];
                fr[x] = 128 * TKS * nst - 8 * (p + q); // row part of the Re correction
                fi[x] = -8 * (q - p);                  // row part of the Im correction
            }
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int32_t p = f8t[jp + 32 * y + lc], q = f8t[256 + jp + 32 * y + lc];
                gr[y] = -8 * (p + q);
                gi[y] = 8 * (q - p);
            }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // one group of rows at a time (keeps the scheduler from
                // hoisting every group's loads and offsets)
                __builtin_amdgcn_sched_barrier(0);
                uint32_t off[4][2];
                int32_t sv[4], cr[4], ci[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = 8 * q + 4 * lh + e;
                    const int i = I0 + ro.ipos[x] + rr;
                    const int rel = (int)((int64_t)i * (i + 1) / 2 - rb0);
                    sv[e] = FUSE ? __shfl(S[x], rr) : 0;
                    cr[e] = ENG == ENG_F8 ? __shfl(fr[x], rr) : 0;
                    ci[e] = ENG == ENG_F8 ? __shfl(fi[x], rr) : 0;
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const int j = J0 + ro.jpos[y] - cofs + lc;
                        off[e][y] = (((own >> (x + 2 * y)) & 1) && i < N && j <= i) ? (uint32_t)(rel + j) * 8u : OOR;
                    }
                }
                u32x2 old[4][2];
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        old[e][y] = add ? __builtin_amdgcn_raw_buffer_load_b64(srs, (int)off[e][y], 0, 0)
                                        : u32x2{0u, 0u};
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const u32x2 v = {old[e][y].x + acc_word<IN_BITS>(accR[x][y][4 * q + e]) +
                                             (uint32_t)(cr[e] + gr[y]),
                                         old[e][y].y + acc_word<IN_BITS>(accI[x][y][4 * q + e]) +
                                             (uint32_t)(sv[e] + ci[e] + gi[y])};
                        __builtin_amdgcn_raw_buffer_store_b64(v, drs, (int)off[e][y], 0, 0);
                    }
            }
        // drain the flush (stores may complete out of order with the copies)
        dma_wait<0>();
    }
}

} // namespace xeng
