// Small-N X-engine kernel (4-bit input, int8 engine, N <= 64 with N a
// multiple of 16): the regime where the samples, not the MFMAs, bound the
// work (N^2 / 2 cells per channel against N bytes per sample).
//
// One work item is one channel of one subarray: V[f] = sum_t x x^H over
// the launch's segment (Section 2.5). The channel's 64 inputs (zero-padded
// past N) form three 32 x 32 MFMA blocks of the lower triangle: the
// diagonal blocks D0 = (0, 0), D1 = (1, 1) and the lower block L = (1, 0).
// Persistent workgroups of 4 waves walk their own slice of the channel list.
//
// Staging: a stage is 256 time rows of the channel's 64 bytes (16 KB),
// copied raw from HBM into a 4-deep LDS ring by buffer loads that write LDS
// directly, 3 stages ahead, as in the 128 x 128 kernel. Within a row the four
// 16-byte chunks sit in slots c ^ 2 ((tau >> 2) & 1), so that the 8 rows x
// 2 chunks of one half-wave transposing read cover all 64 banks.
//
// Work split: the 8 K steps (32 samples) of a stage are dealt to the waves
// round-robin (wave w takes steps w and w + 4); every wave computes all
// three blocks for its steps. The I and J operands of a channel are the
// same samples, so a K step reads and unpacks just two 32-input fragments
// (re, im, ~im of each) for 12 MFMAs, and every wave has the same work
// whichever SIMD it shares with the other workgroup.
//
// End of a channel: the copies are drained, the four waves' partial sums
// are added through the (then idle) LDS ring, and waves 0, 1, 2 write D0, L
// and D1. Sums are raw as in the 128 x 128 kernel (Im V_ij - S_i, the
// diagonal holding -S_i): a flush adds them to `src` (or to nothing) and
// writes `dst`. With FUSE the flush writes exact sums instead, taking S_i
// from the diagonal of the summed D blocks, so no separate row sums are
// needed.
#pragma once

#include "xcorr_wg.h"

namespace xeng {

constexpr int SN_ROWB = 64;                       // bytes per staged row (64 inputs)
constexpr int SN_TKS = WG_STAGE / SN_ROWB;        // time rows per stage (256)
constexpr int SN_KS = SN_TKS / 32;                // K steps per stage (8)
constexpr int SN_NBUF = 4;                        // ring depth (5 measured slower)
constexpr int SN_DMA = WG_STAGE / (WG_THREADS * 16); // 16-byte copies per thread per stage (4)
constexpr int SN_MAX_N = 64;

__device__ __forceinline__ int sn_slot(int tau, int c) { return c ^ (((tau >> 2) & 1) << 1); }

// raw fragments of one wave's two K steps of a stage: [step][row block][load]
typedef i32x2 SnRaw[2][2][2];

struct SnOps {
    i32x4 re[2], im[2], ni[2]; // per 32-input block: re, im, ~im (4-bit values scaled by 16)
};

__device__ __forceinline__ void sn_unpack(const SnRaw &R, int k, SnOps &o)
{
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const u32x4 p = {(uint32_t)R[k][b][0].x, (uint32_t)R[k][b][0].y, (uint32_t)R[k][b][1].x,
                         (uint32_t)R[k][b][1].y};
        const u32x4 im = (p << 4) & 0xF0F0F0F0u;
        o.re[b] = (i32x4)(p & 0xF0F0F0F0u);
        o.im[b] = (i32x4)im;
        o.ni[b] = (i32x4)(im ^ 0xF0F0F0F0u);
    }
}

// Block q of the channel: 0 = D0 (rows 0.., cols 0..), 1 = L (rows 32..,
// cols 0..), 2 = D1 (rows 32.., cols 32..).
//   accR += re_I re_J + im_I im_J,  accI += re_I ~im_J + im_I re_J.
__device__ __forceinline__ void sn_mfma(const SnOps &o, i32x16 (&accR)[3], i32x16 (&accI)[3])
{
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int x = q == 0 ? 0 : 1, y = q == 2 ? 1 : 0;
        accR[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.re[x], o.re[y], accR[q], 0, 0, 0);
        accI[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.re[x], o.ni[y], accI[q], 0, 0, 0);
        accR[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.im[x], o.im[y], accR[q], 0, 0, 0);
        accI[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.im[x], o.re[y], accI[q], 0, 0, 0);
    }
}

template <bool FUSE>
__global__ __launch_bounds__(WG_THREADS, 2) void xcorr_sn_kernel(WgArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[SN_NBUF * WG_STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    typedef __attribute__((address_space(4))) const uint32_t c_u32_t;
    typedef __attribute__((address_space(4))) const int32_t c_i32_t;
    c_u32_t *itw = (c_u32_t *)a.items;
    c_i32_t *wbeg = (c_i32_t *)a.wg_begin;
    const int it_begin = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x]);
    const int it_end = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x + 1]);
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    constexpr uint32_t OOR = 0x80000000u;

    // transposing-read offsets of this lane (see xcorr_wg.h for the lane
    // pattern of ds_read_b64_tr_b8): load i of row block b of K step k of a
    // stage sits at fo[b] + (32 k + 8 i) * SN_ROWB
    const int G = lane >> 4;
    int fo[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int m = (lane >> 1) & 7, h = lane & 1;
        const int tau = 16 * (G >> 1) + m;
        const int c = 2 * b + (G & 1);
        fo[b] = tau * SN_ROWB + 16 * sn_slot(tau, c) + 8 * h;
    }

    for (int it = it_begin; it < it_end; ++it) {
        const int u = __builtin_amdgcn_readfirstlane(it);
        const uint32_t cs = itw[2 * u];
        const WgSub &sb = a.subs[cs >> 24];
        const int f = (int)(cs & 0xFFFFFFu);
        const int N = sb.n_inputs;
        const uint32_t rowstride = (uint32_t)sb.n_chans * (uint32_t)N;
        const int tcount = sb.t_count;
        const int nst = (tcount + SN_TKS - 1) / SN_TKS;
        const uint8_t *base = sb.samples + ((size_t)sb.t_begin * sb.n_chans + f) * (size_t)N;

        // this thread's copies: stage position P = k * 256 + tid (16 bytes
        // each) is row P / 4, slot P % 4, which holds chunk sn_slot(row, slot)
        uint32_t voff[SN_DMA];
#pragma unroll
        for (int k = 0; k < SN_DMA; ++k) {
            const int P = k * WG_THREADS + tid;
            const int tau = P >> 2, sl = P & 3;
            const int c = sn_slot(tau, sl); // the swizzle is its own inverse
            voff[k] = 16 * c < N ? (uint32_t)tau * rowstride + (uint32_t)(16 * c) : OOR;
        }
        int issued = 0;
        auto issue = [&]() {
            const int t_first = issued * SN_TKS;
            const int nt = tcount - t_first < SN_TKS ? tcount - t_first : SN_TKS;
            const uint64_t gb = (uint64_t)(uintptr_t)(base + (size_t)t_first * rowstride);
            const i32x4 rsrc = {(int)(uint32_t)gb, (int)((uint32_t)(gb >> 32) & 0xFFFFu),
                                (int)((uint32_t)nt * rowstride), 0x00020000};
            const uint32_t dst = lds_base + (uint32_t)((issued % SN_NBUF) * WG_STAGE + wave * 1024);
#pragma unroll
            for (int k = 0; k < SN_DMA; ++k) dma16(rsrc, voff[k], dst + (uint32_t)(k * WG_THREADS * 16));
            ++issued;
        };
        // stage s visible to every wave: this wave's copies of it landed
        // (at most the later stages outstanding), then barrier; rows past the
        // segment's end cleared
        auto prep = [&](int s) {
            const int later = issued - (s + 1);
            if (later >= SN_NBUF - 2) wg_wait_barrier(SN_NBUF - 2);
            else if (later >= 1) wg_wait_barrier(1);
            else wg_wait_barrier(0);
            const int nt = tcount - s * SN_TKS;
            if (nt < SN_TKS) {
                uint8_t *b = lds + (s % SN_NBUF) * WG_STAGE;
                for (int o = tid * 16; o < WG_STAGE; o += WG_THREADS * 16)
                    if (o / SN_ROWB >= nt) *(u32x4 *)(b + o) = u32x4{0u, 0u, 0u, 0u};
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            }
        };
        // this wave's K steps (wave and wave + 4) of stage s
        auto read = [&](int s, SnRaw &R) {
            const uint8_t *b = lds + (s % SN_NBUF) * WG_STAGE;
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int blk = 0; blk < 2; ++blk)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        R[k][blk][i] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                            (lds_i32x2 *)(b + fo[blk] + (32 * (wave + 4 * k) + 8 * i) * SN_ROWB));
        };

        i32x16 accR[3], accI[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            accR[q] = i32x16{};
            accI[q] = i32x16{};
        }
#pragma unroll
        for (int k = 0; k < SN_NBUF - 1; ++k)
            if (issued < nst) issue();
        SnRaw R;
        SnOps O0, O1;
        prep(0);
        read(0, R);
        for (int s = 0; s < nst; ++s) {
            // the slot of stage s - 1 is free: every wave read it before the
            // barrier that published stage s
            if (issued < nst) issue();
            sn_unpack(R, 0, O0);
            sn_unpack(R, 1, O1);
            if (s + 1 < nst) {
                prep(s + 1);
                read(s + 1, R);
            }
            sn_mfma(O0, accR, accI);
            sn_mfma(O1, accR, accI);
        }

        // ---- reduction of the four waves' sums through the drained ring.
        // Region A (32 KB) holds D1 then D0, region B holds L; each wave's
        // 32 accumulator registers (16 Re, 16 Im) of a block take 8 KB,
        // stored as 32 dwords per lane in lane-major 16-byte groups.
        dma_wait<0>();
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        auto put = [&](int region, int q) {
            u32x4 *d = (u32x4 *)(lds + region + wave * 8192) + lane;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                d[64 * g] = u32x4{(uint32_t)accR[q][4 * g], (uint32_t)accR[q][4 * g + 1],
                                  (uint32_t)accR[q][4 * g + 2], (uint32_t)accR[q][4 * g + 3]};
                d[64 * (4 + g)] = u32x4{(uint32_t)accI[q][4 * g], (uint32_t)accI[q][4 * g + 1],
                                        (uint32_t)accI[q][4 * g + 2], (uint32_t)accI[q][4 * g + 3]};
            }
        };
        auto gather = [&](int region, int q) {
#pragma unroll
            for (int w = 1; w < 4; ++w) {
                const u32x4 *d = (const u32x4 *)(lds + region + ((wave + w) & 3) * 8192) + lane;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const u32x4 r = d[64 * g], i = d[64 * (4 + g)];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        accR[q][4 * g + e] += (int32_t)r[e];
                        accI[q][4 * g + e] += (int32_t)i[e];
                    }
                }
            }
        };
        constexpr int RA = 0, RB = 2 * 16384, RS = 3 * 16384 + 8192; // RS: D1's diagonal (32 words)
        put(RA, 2);
        put(RB, 1);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (wave == 2) gather(RA, 2);
        if (wave == 1) gather(RB, 1);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        put(RA, 0);
        // 32 x 32 MFMA result layout: lane l holds column l % 32 of rows
        // 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15; the diagonal cell of
        // row rr sits in lane rr + 32 (rr / 4 % 2)
        const int lh = lane >> 5, lc = lane & 31;
        if (wave == 2) {
            // D1's diagonal words: -S_i of rows 32..63 (this launch's part)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rr = 8 * (r >> 2) + 4 * lh + (r & 3);
                if (lc == rr) *(int32_t *)(lds + RS + 4 * rr) = accI[2][r];
            }
        }
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (wave == 0) gather(RA, 0);

        // ---- flush: wave 0 writes D0, wave 1 L, wave 2 D1. Lane-derived
        // offsets come from an opaque copy of the lane index, so that they are
        // not hoisted out of the channel loop (and kept live across it).
        int fl = lane;
        asm volatile("" : "+v"(fl));
        const int fh = fl >> 5, fc = fl & 31;
        auto flush = [&](const i32x16 &bR, const i32x16 &bI, const int q) {
            const int r0 = q == 0 ? 0 : 32, c0 = q == 2 ? 32 : 0;
            if (r0 >= N) return;
            // this launch's -S_i of each row this lane holds: the diagonal
            // of the wave's own block, or D1's (for L) from LDS
            int32_t sv[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rr = 8 * (r >> 2) + 4 * fh + (r & 3);
                if (!FUSE) sv[r] = 0;
                else if (q == 1) sv[r] = *(const int32_t *)(lds + RS + 4 * rr);
                else sv[r] = __shfl(bI[r], rr + 32 * fh);
            }
            const int64_t tri = (int64_t)N * (N + 1) / 2;
            const int rlim = r0 + 32 < N ? r0 + 32 : N;
            const int64_t rb0 = (int64_t)r0 * (r0 + 1) / 2;
            const int64_t rb1 = (int64_t)rlim * (rlim + 1) / 2;
            const size_t cell0 = (size_t)f * (size_t)tri + (size_t)rb0;
            const int nbytes = (int)((rb1 - rb0) * 8);
            const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)((uint2 *)sb.dst + cell0), (short)0, nbytes, 0x00020000);
            const bool add = sb.src != nullptr;
            const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)((const uint2 *)(add ? sb.src : sb.dst) + cell0), (short)0, add ? nbytes : 0,
                0x00020000);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rr = 8 * (r >> 2) + 4 * fh + (r & 3);
                const int i = r0 + rr, j = c0 + fc;
                const int rel = (int)((int64_t)i * (i + 1) / 2 - rb0);
                const uint32_t off = (i < N && j <= i) ? (uint32_t)(rel + j) * 8u : OOR;
                u32x2 old = {0u, 0u};
                int32_t sd = 0;
                if (add) {
                    old = __builtin_amdgcn_raw_buffer_load_b64(srs, (int)off, 0, 0);
                    if (FUSE) {
                        // src's own diagonal word of row i (its -S_i in the raw form)
                        const uint32_t doff = i < N ? (uint32_t)(rel + i) * 8u : OOR;
                        const u32x2 dg = __builtin_amdgcn_raw_buffer_load_b64(srs, (int)doff, 0, 0);
                        sd = (int32_t)dg.y;
                    }
                }
                const u32x2 v = {old.x + acc_word<4>(bR[r]),
                                 old.y + acc_word<4>(bI[r]) - (uint32_t)sd - acc_word<4>(sv[r])};
                __builtin_amdgcn_raw_buffer_store_b64(v, drs, (int)off, 0, 0);
            }
        };
        if (wave == 0) flush(accR[0], accI[0], 0);
        else if (wave == 1) flush(accR[1], accI[1], 1);
        else if (wave == 2) flush(accR[2], accI[2], 2);
        // the ring is reused by the next channel's copies: every wave is done
        // with the reduction regions
        dma_wait<0>();
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }
}

} // namespace xeng
