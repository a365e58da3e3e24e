// X-engine tile kernel: int8 MFMA, int32 accumulation, gfx950 (CDNA4).
//
// One workgroup computes one (channel, I-block, J-block) tile of the lower
// triangle of V[f] = sum_t x(t, f) x(t, f)^H (Section 2.5; Fig. 2 caption),
// with J-block <= I-block, for the samples of one time segment.
//
// Data flow per stage of TK = 64 time samples:
//   1. every thread loads 16 time rows x 4 inputs (one dword per row) of the
//      [T][F][N] stream: each wave instruction reads 256 contiguous bytes;
//   2. a 4x4 byte transpose in registers (v_perm) turns them into 4 inputs x
//      16 consecutive time samples, written to LDS as packed rows
//      [row][time] (1 byte per complex sample), double-buffered;
//   3. each wave reads its 16-byte fragments (one input row, 16 samples) and
//      unpacks them with masks only:
//        w & 0xF0F0F0F0        = 16 * re   (high nibble, sign already in bit 7)
//        (w << 4) & 0xF0F0F0F0 = 16 * im
//        16*im ^ 0xF0F0F0F0    = 16 * (~im) = 16 * (-im - 1)
//      (the negated operand uses ~im, not -im: -(-8 * 16) would leave int8);
//   4. four v_mfma_i32_16x16x64_i8 per 16x16 sub-tile and stage:
//        accR += (16re_i)(16re_j) + (16im_i)(16im_j)             = 256 Re V
//        accI += (16re_i)(16(~im_j)) + (16im_i)(16re_j)          = 256 (Im V - S_i)
//      with S_i = sum_t re_i(t). The accumulator keeps this raw form. Since
//      Im V_ii = 0, the diagonal cell holds -S_i exactly, and the dump
//      kernel recovers Im V_ij = raw_ij - raw_ii (mod 2^32, exact).
// For 8+8-bit input the rows hold int8 re and im separately (no scaling) and
// the same ~im identity gives accI = Im V - S_i.
//
// Exactness: every quantity is an integer; int32 MFMA sums wrap modulo 2^32
// but each segment is at most SEG_T = 32768 samples, so the final 256 Re V and
// 256 (Im V - S_i) of a segment stay inside int32 (|Re V|, |Im V| <= 128 T for
// 4-bit; <= 32768 T unscaled for 8-bit) and the shifts back are exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int TK = 64;          // time samples per LDS stage
constexpr int SEG_T = 32768;    // most samples one launch may integrate
constexpr int WG_THREADS = 256; // 4 waves in a 2 x 2 grid of wave tiles

struct TileArgs {
    const uint8_t *samples; // [T][F][N] (4-bit) or [T][F][N][2] (8-bit)
    int32_t *vis;           // [F][tri(N)][2]
    int64_t t_begin;        // first sample of this segment
    int32_t t_count;        // samples in this segment (<= SEG_T)
    int32_t n_chans;
    int32_t n_inputs;
    int32_t n_tiles;        // tiles per channel: nb (nb + 1) / 2
    int32_t n_work;         // n_tiles * n_chans = grid size
    int32_t accumulate;     // 0: overwrite the accumulator, 1: add to it
};

// Byte transpose of a 4x4 block held in 4 dwords: in[s] byte q -> out[q] byte s.
__device__ __forceinline__ void transpose4x4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                             uint32_t &o0, uint32_t &o1, uint32_t &o2,
                                             uint32_t &o3)
{
    // __builtin_amdgcn_perm(hi, lo, sel): byte k of the result is byte sel[k]
    // of the 8-byte value {hi:lo} (bytes 0-3 from lo, 4-7 from hi).
    const uint32_t lo_ab = __builtin_amdgcn_perm(b, a, 0x05010400u); // a0 b0 a1 b1
    const uint32_t hi_ab = __builtin_amdgcn_perm(b, a, 0x07030602u); // a2 b2 a3 b3
    const uint32_t lo_cd = __builtin_amdgcn_perm(d, c, 0x05010400u); // c0 d0 c1 d1
    const uint32_t hi_cd = __builtin_amdgcn_perm(d, c, 0x07030602u); // c2 d2 c3 d3
    o0 = __builtin_amdgcn_perm(lo_cd, lo_ab, 0x05040100u);           // a0 b0 c0 d0
    o1 = __builtin_amdgcn_perm(lo_cd, lo_ab, 0x07060302u);           // a1 b1 c1 d1
    o2 = __builtin_amdgcn_perm(hi_cd, hi_ab, 0x05040100u);           // a2 b2 c2 d2
    o3 = __builtin_amdgcn_perm(hi_cd, hi_ab, 0x07060302u);           // a3 b3 c3 d3
}

// Map a linear workgroup id so that the workgroups one XCD runs (ids
// congruent mod 8, dispatched round-robin over the 8 XCDs) get consecutive
// work items, i.e. the tiles of the same channels, which share input rows in
// that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    const int per = n / 8, rem = n % 8;
    const int x = bid % 8, k = bid / 8;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

// Tile index t of the lower block triangle -> (bi, bj), bj <= bi, row-major.
__device__ __forceinline__ void tri_decode(int t, int &bi, int &bj)
{
    int i = (int)((__builtin_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    bi = i;
    bj = t - i * (i + 1) / 2;
}

// Swizzle of the 16-byte time slots of a staged row, so that 8 lanes reading
// the same slot of 8 consecutive rows touch 8 different bank groups.
__device__ __forceinline__ int slot_swz(int row) { return (row >> 1) & 3; }

// IN_BITS = 4: staged row = TK bytes (packed samples).
// IN_BITS = 8: two staged rows per input (re row, im row), TK bytes each.
// WT = wave tile edge in 16-row sub-blocks; workgroup tile edge BT = 32 * WT.
template <int IN_BITS, int WT, bool ALIGNED>
__global__ __launch_bounds__(WG_THREADS, (IN_BITS == 8 && WT == 4) ? 1 : 2) void xcorr_i8_kernel(TileArgs a)
{
    constexpr int BT = 32 * WT;            // workgroup tile edge (inputs)
    constexpr int HB = BT / 2;             // wave tile edge
    constexpr int NROW = 2 * BT;           // staged inputs: I block then J block
    constexpr int RPI = IN_BITS == 4 ? 1 : 2;  // staged rows per input
    constexpr int ROWB = TK;               // bytes per staged row per stage
    constexpr int BUF = NROW * RPI * ROWB; // bytes per stage buffer
    // staging units: groups of 4 (4-bit) or 2 (8-bit) inputs x 16 time samples
    constexpr int IPU = IN_BITS == 4 ? 4 : 2;
    constexpr int NGRP = NROW / IPU;
    constexpr int NUNIT = NGRP * (TK / 16);
    constexpr int UPT = (NUNIT + WG_THREADS - 1) / WG_THREADS; // units per thread

    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * BUF];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    const int work = xcd_remap(blockIdx.x, a.n_work);
    const int f = work / a.n_tiles;
    int bi, bj;
    tri_decode(work - f * a.n_tiles, bi, bj);
    const int I0 = bi * BT, J0 = bj * BT;
    const bool diag = bi == bj;
    const int N = a.n_inputs;
    const int F = a.n_chans;
    // a wave whose whole tile lies above the diagonal has nothing to compute
    const bool active = !(diag && wr < wc);

    // ---- staging assignment (fixed over the time loop)
    constexpr int SB = IN_BITS == 4 ? 1 : 2;            // bytes per complex sample
    const size_t row_stride = (size_t)F * N * SB;       // bytes per time step
    bool u_on[UPT];
    int u_blk[UPT], u_row0[UPT], u_gin[UPT];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const int unit = tid + u * WG_THREADS;
        u_on[u] = unit < NUNIT;
        const int grp = unit % NGRP;
        u_blk[u] = unit / NGRP;                          // 16-sample block of the stage
        u_row0[u] = grp * IPU;                           // first staged input of the group
        u_gin[u] = u_row0[u] < BT ? I0 + u_row0[u] : J0 + (u_row0[u] - BT);
    }

    // Staging loads are raw buffer loads with a descriptor per stage whose
    // range ends at the last valid sample of the segment: reads past it, and
    // reads of lanes whose inputs lie past N (given an out-of-range offset),
    // return 0 without any branch, so every load of a stage is in flight at
    // once. Offsets are 32-bit relative to the stage's first row (the host
    // checks that a stage spans less than 2^31 bytes). Inputs that do not
    // fill whole dwords (ALIGNED == false) are loaded byte by byte.
    constexpr uint32_t OOR = 0x80000000u;    // offset beyond any stage range
    uint32_t u_voff[UPT];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const bool in_ok = u_on[u] && u_gin[u] + IPU <= N;
        u_voff[u] = (ALIGNED && !in_ok) || !u_on[u]
                        ? OOR
                        : (uint32_t)(u_blk[u] * 16) * (uint32_t)row_stride + (uint32_t)(u_gin[u] * SB);
    }

    auto load_stage = [&](int stage, uint32_t (&d)[UPT][16]) {
        const int t_first = stage * TK;
        const int nt = a.t_count - t_first < TK ? a.t_count - t_first : TK;
        const uint8_t *base = a.samples + ((size_t)(a.t_begin + t_first) * F + f) * (size_t)N * SB;
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)base, (short)0, (int)((uint32_t)nt * (uint32_t)row_stride), 0x00020000);
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const uint32_t off = u_voff[u] + (uint32_t)s * (uint32_t)row_stride;
                if (ALIGNED) {
                    d[u][s] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off, 0, 0);
                } else {
                    uint32_t v = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int in = u_gin[u] + (IN_BITS == 4 ? b : b / 2);
                        const uint32_t ob = (u_on[u] && in < N) ? off + (uint32_t)b : OOR;
                        v |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rsrc, (int)ob, 0, 0) << (8 * b);
                    }
                    d[u][s] = v;
                }
            }
        }
    };

    auto store_stage = [&](uint8_t *buf, const uint32_t (&d)[UPT][16]) {
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            if (!u_on[u]) continue;
            uint32_t e[4][4]; // e[q][c]: byte column q of 4x4 block c
#pragma unroll
            for (int c = 0; c < 4; ++c)
                transpose4x4(d[u][4 * c], d[u][4 * c + 1], d[u][4 * c + 2], d[u][4 * c + 3],
                             e[0][c], e[1][c], e[2][c], e[3][c]);
            // 4-bit: byte q of a dword is input row0 + q.
            // 8-bit: byte q is (input row0 + q/2, re if q even else im).
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = IN_BITS == 4 ? u_row0[u] + q : 2 * (u_row0[u] + q / 2) + (q & 1);
                const int slot = u_blk[u] ^ slot_swz(row);
                u32x4 v = {e[q][0], e[q][1], e[q][2], e[q][3]};
                *(u32x4 *)(buf + row * ROWB + slot * 16) = v;
            }
        }
    };

    i32x4 accR[WT][WT], accI[WT][WT];
#pragma unroll
    for (int x = 0; x < WT; ++x)
#pragma unroll
        for (int y = 0; y < WT; ++y) {
            accR[x][y] = i32x4{0, 0, 0, 0};
            accI[x][y] = i32x4{0, 0, 0, 0};
        }

    const int nstage = (a.t_count + TK - 1) / TK;
    const int kg = lane >> 4;   // k-group: samples 16 kg .. 16 kg + 15 of a stage
    const int lr = lane & 15;   // row within a 16-row sub-block

    uint32_t d[UPT][16];
    load_stage(0, d);
    store_stage(lds, d);
    __syncthreads();

    for (int st = 0; st < nstage; ++st) {
        const uint8_t *buf = lds + (st & 1) * BUF;
        if (st + 1 < nstage) load_stage(st + 1, d);

        if (active) {
            i32x4 reI[WT], imI[WT];
#pragma unroll
            for (int x = 0; x < WT; ++x) {
                const int in = wr * HB + 16 * x + lr;           // staged input (I block)
                if (IN_BITS == 4) {
                    const u32x4 p = *(const u32x4 *)(buf + in * ROWB + ((kg ^ slot_swz(in)) * 16));
                    reI[x] = (i32x4)(p & 0xF0F0F0F0u);
                    imI[x] = (i32x4)((p << 4) & 0xF0F0F0F0u);
                } else {
                    const int rr = 2 * in, ri = 2 * in + 1;
                    reI[x] = *(const i32x4 *)(buf + rr * ROWB + ((kg ^ slot_swz(rr)) * 16));
                    imI[x] = *(const i32x4 *)(buf + ri * ROWB + ((kg ^ slot_swz(ri)) * 16));
                }
            }
#pragma unroll
            for (int y = 0; y < WT; ++y) {
                const int in = BT + wc * HB + 16 * y + lr;      // staged input (J block)
                i32x4 reJ, imJ, niJ;
                if (IN_BITS == 4) {
                    const u32x4 p = *(const u32x4 *)(buf + in * ROWB + ((kg ^ slot_swz(in)) * 16));
                    const u32x4 im = (p << 4) & 0xF0F0F0F0u;
                    reJ = (i32x4)(p & 0xF0F0F0F0u);
                    imJ = (i32x4)im;
                    niJ = (i32x4)(im ^ 0xF0F0F0F0u);
                } else {
                    const int rr = 2 * in, ri = 2 * in + 1;
                    reJ = *(const i32x4 *)(buf + rr * ROWB + ((kg ^ slot_swz(rr)) * 16));
                    imJ = *(const i32x4 *)(buf + ri * ROWB + ((kg ^ slot_swz(ri)) * 16));
                    niJ = ~imJ;
                }
#pragma unroll
                for (int x = 0; x < WT; ++x) {
                    accR[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(reI[x], reJ, accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(reI[x], niJ, accI[x][y], 0, 0, 0);
                    accR[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(imI[x], imJ, accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(imI[x], reJ, accI[x][y], 0, 0, 0);
                }
            }
        }

        if (st + 1 < nstage) store_stage(lds + ((st + 1) & 1) * BUF, d);
        __syncthreads();
    }

    if (!active) return;

    // ---- flush: 16x16 MFMA result layout, lane holds column (lane & 15) of
    // rows 4 (lane >> 4) + r, r = 0..3
    const int64_t tri = (int64_t)N * (N + 1) / 2;
    uint2 *vis = (uint2 *)a.vis + (size_t)f * (size_t)tri;
#pragma unroll
    for (int x = 0; x < WT; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rl = wr * HB + 16 * x + 4 * kg + r;
            const int i = I0 + rl;
            if (i >= N) continue;
            const int64_t rowbase = (int64_t)i * (i + 1) / 2;
#pragma unroll
            for (int y = 0; y < WT; ++y) {
                const int j = J0 + wc * HB + 16 * y + lr;
                if (j > i) continue;
                // raw convention: Im holds Im V - S_i, corrected at the dump
                const uint32_t re = (uint32_t)(IN_BITS == 4 ? accR[x][y][r] >> 8 : accR[x][y][r]);
                const uint32_t im = (uint32_t)(IN_BITS == 4 ? accI[x][y][r] >> 8 : accI[x][y][r]);
                uint2 *p = vis + rowbase + j;
                if (a.accumulate) {
                    const uint2 o = *p;
                    *p = make_uint2(o.x + re, o.y + im);
                } else {
                    *p = make_uint2(re, im);
                }
            }
        }
}

// Clear n int32 words (used instead of a memset so that the work can sit in a
// captured graph).
__global__ void fill_zero_kernel(int4 *p, size_t n16, int32_t *tail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        p[k] = make_int4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}


// Fast-cadence autocorrelations (Section 2.6: the autocorrelations of chosen
// inputs are dumped and zeroed more often than the cross power, by selective
// dumping and zeroing of accumulator cells). out[f][q] = Re V_ii of input
// i = inputs[q] in channel f (Im V_ii is identically 0); reset clears only
// that Re word: the diagonal's Im word holds -S_i, which the dump of every
// cross cell of row i needs for the whole integration. One thread per
// (channel, selected input), grid-stride.
__global__ __launch_bounds__(256) void fast_autos_kernel(uint2 *__restrict__ acc, int64_t tri,
                                                         int32_t n_chans,
                                                         const int32_t *__restrict__ inputs,
                                                         int32_t n, int32_t *__restrict__ out,
                                                         int32_t reset, int32_t acc_zero)
{
    const int64_t total = (int64_t)n_chans * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = e / n;
        const int64_t i = inputs[e - f * n];
        const int64_t c = f * tri + i * (i + 1) / 2 + i;
        if (out) out[e] = acc_zero ? 0 : (int32_t)acc[c].x;
        if (reset && !acc_zero) acc[c].x = 0u;
    }
}

// Dump of a raw accumulator into the output convention: Re unchanged,
// Im V_ij = raw_ij - raw_ii (the diagonal entry of row i holds -S_i).
// Arithmetic is modulo 2^32; the true value fits int32.
//
// Grid: (ceil(tri / DUMP_PER_WG), channels), starting at channel chan0. Each
// workgroup converts DUMP_PER_WG consecutive cells of one channel; every load and store
// instruction of a wave covers 64 consecutive 8-byte cells. The row index of
// cell k solves i (i + 1) / 2 <= k < (i + 1) (i + 2) / 2: a float square root
// gives it to within one, and one integer correction each way makes it exact
// (k < 2^31, so 8k + 1 is off by at most 2^7 in float and its root by less
// than 2^-8).
constexpr int DUMP_ITEMS = 8;
constexpr int DUMP_PER_WG = 256 * DUMP_ITEMS;

__global__ __launch_bounds__(256) void dump_kernel(const uint2 *__restrict__ acc,
                                                   uint2 *__restrict__ out, int32_t tri,
                                                   int32_t chan0)
{
    const int64_t cbase = (int64_t)(chan0 + blockIdx.y) * tri;
    const int32_t k0 = blockIdx.x * DUMP_PER_WG + threadIdx.x;
    uint2 v[DUMP_ITEMS];
    uint32_t sd[DUMP_ITEMS];
#pragma unroll
    for (int r = 0; r < DUMP_ITEMS; ++r) {
        const int32_t k = k0 + 256 * r;
        if (k < tri) v[r] = acc[cbase + k];
    }
#pragma unroll
    for (int r = 0; r < DUMP_ITEMS; ++r) {
        const int32_t k = k0 + 256 * r;
        if (k < tri) {
            int64_t i = (int64_t)((__builtin_sqrtf(8.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
            if (i * (i + 1) / 2 > k) --i;
            if ((i + 1) * (i + 2) / 2 <= k) ++i;
            sd[r] = acc[cbase + i * (i + 1) / 2 + i].y;
        }
    }
#pragma unroll
    for (int r = 0; r < DUMP_ITEMS; ++r) {
        const int32_t k = k0 + 256 * r;
        if (k < tri) out[cbase + k] = make_uint2(v[r].x, v[r].y - sd[r]);
    }
}

// The LDS DMA is issued from inline assembly so that the compiler does not
// see an asynchronous LDS write: left to itself it waits for every
// outstanding DMA (vmcnt(0)) before any LDS read and at every barrier, which
// would drain the ring each stage. The kernel counts the outstanding DMAs of
// each wave itself (every wave issues exactly LPS of them per stage, lanes
// without data get an out-of-range offset instead of an exec mask, so the
// count never varies).
//
// One 16-byte buffer load per lane into LDS: lane l's 16 bytes land at
// lds_addr + 16 l (lds_addr must be wave-uniform).
__device__ __forceinline__ void dma16(i32x4 rsrc, uint32_t voff, uint32_t lds_addr)
{
    // the descriptor and the LDS address are wave-uniform; make that explicit
    const i32x4 sr = {__builtin_amdgcn_readfirstlane(rsrc.x), __builtin_amdgcn_readfirstlane(rsrc.y),
                      __builtin_amdgcn_readfirstlane(rsrc.z), __builtin_amdgcn_readfirstlane(rsrc.w)};
    asm volatile("s_mov_b32 m0, %2\n\t"
                 "s_nop 0\n\t"
                 "buffer_load_dwordx4 %0, %1, 0 offen lds"
                 :
                 : "v"(voff), "s"(sr), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
                 : "memory");
}

// Wait until at most N of this wave's vector-memory operations are
// outstanding. The memory clobber keeps the compiler from moving LDS
// accesses across the wait.
template <int N>
__device__ __forceinline__ void dma_wait()
{
    asm volatile("s_waitcnt vmcnt(%0)" : : "n"(N) : "memory");
}

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) i32x2 lds_i32x2;

} // namespace xeng
