// Wave-private X-engine kernels for 4-bit input (N a multiple of 16), int8
// MFMA with int32 accumulation, in two shapes:
//   V = 1: one wave per SIMD (up to 512 registers: 8 accumulator blocks of
//          32 x 32, 256 accumulation registers), items of 128 x 64;
//   V = 2: two waves per SIMD (256 registers each: 4 accumulator blocks),
//          items of 64 x 64; the two waves of a SIMD fill each other's issue
//          gaps around the matrix core.
//
// Work is a host-built list of items of the lower block triangle of
// V[f] = sum_t x(t, f) x(t, f)^H (Section 2.5; Fig. 2 caption), over square
// tiles (channel f, input block I, block J <= I) of 128 (V = 1) or 64 (V = 2)
// inputs:
//   - V = 1: an off-diagonal tile is two items, one per 64-input half h of
//     its J block (4 x 2 MFMA blocks); a diagonal tile's 10 blocks on or
//     below the diagonal are split into two items of 5, part 0 =
//     (0,0) (1,0) (2,0) (3,0) (1,1) and part 1 = (2,1) (3,1) (2,2) (3,2) (3,3)
//     (x = I block, y = J block of 32 inputs);
//   - V = 2: an off-diagonal tile is one item (2 x 2 blocks); a diagonal
//     tile is one item of its 3 blocks (0,0) (1,0) (1,1).
// No block above the diagonal is computed. Every workgroup is one wave and
// walks its own slice of the list.
//
// Staging: every wave owns an LDS ring of 32-sample stages (one K step of
// v_mfma_i32_32x32x32_i8). A stage is an I region (32 rows x the item's I
// inputs) and a J region (32 rows x its J inputs), copied raw from HBM by
// buffer loads that write LDS directly, NBUF - 1 stages ahead of the one
// being multiplied. Nothing is shared between waves, so there are no
// barriers: a wave only waits for its own copies. Copies are issued past the
// end of the list too (out of range, no memory traffic), so every wait on
// them is the same.
//
// Fragments: as in the persistent 4-wave kernel, ds_read_b64_tr_b8 turns the
// time-major rows into the K-major operands (lane l: input l % 32, K group
// l / 32). Chunk c (16 inputs) of row tau sits in slot c ^ (tau & 7) of a
// 128-byte row and in slot c ^ 2 ((tau >> 2) & 1) of a 64-byte row, so the 8
// rows a 16-lane group reads fall on distinct banks. The fragments of stage
// s + 1 are read while stage s is multiplied.
//
// Operands: re = w & 0xF0F0F0F0 and im = (w << 4) & 0xF0F0F0F0 are 16 x the
// nibbles, so products are 256 x the true ones. The imaginary part uses
// ~im = -im - 1 on the J side (so that -(-8) never has to fit in int8):
//   accI = sum re_I ~im_J + im_I re_J = 256 (Im V_ij - S_i),  S_i = sum_t re_i,
// and S_i is summed from the raw bytes by v_dot8_i32_i4 with weights 1 on the
// real nibbles, so the flush writes the exact Im V_ij. Segments of at most
// SEG_T samples keep 256 |sum| <= 2^30.
//
// Flush: each item adds its sums to `src` (the accumulator, when it holds an
// earlier part of the integration) and writes `dst` (the accumulator, or the
// caller's output for a correlate-and-dump), in the output layout
// [F][N(N+1)/2][2]. These kernels always write exact sums (a zero diagonal
// in the raw form of the other kernels, see xcorr_wg.h); src's diagonal word
// of row i is subtracted, so they may also finish an integration begun by
// the other kernels.
#pragma once

#include <type_traits>

#include "xcorr_wg.h"

namespace xeng {

constexpr int W1_TK = 32; // samples per stage (one K step)

// Geometry of the two shapes (bytes per staged row are the input counts).
template <int V> struct W1Geo;
template <> struct W1Geo<1> {
    static constexpr int IB = 128, JB = 64;   // staged I and J inputs
    static constexpr int NBUF = 6;            // stages in a wave's ring
    static constexpr int WG_PER_CU = 4;       // one wave per SIMD
    static constexpr int TILE = 128;          // tile edge of the item list
};
template <> struct W1Geo<2> {
    static constexpr int IB = 64, JB = 64;
    static constexpr int NBUF = 4;
    static constexpr int WG_PER_CU = 8;       // two waves per SIMD
    static constexpr int TILE = 64;
};
template <int V> struct W1Layout {
    typedef W1Geo<V> G;
    static constexpr int JBASE = W1_TK * G::IB;            // J region offset in a stage
    static constexpr int STAGE = W1_TK * (G::IB + G::JB);  // bytes per stage
    static constexpr int DMA = STAGE / (64 * 16);          // 16-byte copies per lane per stage
    static constexpr int IU = JBASE / (64 * 16);           // of which in the I region
    static constexpr int AHEAD = G::NBUF - 1;              // stages copied ahead
};

// Slot of 16-byte chunk c in row tau of a region with `rowb`-byte rows.
__device__ __forceinline__ constexpr int w1_slot(int rowb, int tau, int c)
{
    return rowb == 128 ? c ^ (tau & 7) : c ^ (((tau >> 2) & 1) << 1);
}

struct W1Sub {
    const uint8_t *samples; // [T][F][N] packed 4+4-bit
    const int32_t *src;     // sums to add ([F][tri(N)][2]), or null
    int32_t *dst;           // where the flush writes ([F][tri(N)][2])
    int64_t t_begin;        // first sample of this launch's segment
    int32_t t_count;        // samples in this segment (1 .. SEG_T)
    int32_t n_chans;
    int32_t n_inputs;       // multiple of 16
    int32_t pad;
};

// Item: cs = chan | sub << 24; ij = bi | bj << 12 | role << 24 with role 0, 1
// = off-diagonal tile, J half 0 or 1; 2, 3 = diagonal tile, part 0 or 1.
struct W1Args {
    W1Sub subs[WG_MAX_SUBS];
    const WgItem *items;
    const int32_t *wg_begin; // [n_wg + 1] item ranges per workgroup
};

// Per-role geometry. Read block k is a 32-input block of the stage (region,
// position); MFMA block b multiplies read block xr(b) (I side, rows) by read
// block yr(b) (J side, columns) into output block (ox(b), oy(b)) of 32 x 32
// relative to the item's origin.
template <int V, int R> struct W1Role;

template <> struct W1Role<1, 0> { // off-diagonal half tile: 128 I x 64 J
    static constexpr int NRD = 6, NB = 8;
    __device__ static constexpr bool jreg(int k) { return k >= 4; }
    __device__ static constexpr int pos(int k) { return k < 4 ? 32 * k : 32 * (k - 4); }
    __device__ static constexpr int xr(int b) { return b & 3; }
    __device__ static constexpr int yr(int b) { return 4 + (b >> 2); }
    __device__ static constexpr int ox(int b) { return b & 3; }
    __device__ static constexpr int oy(int b) { return b >> 2; }
    __device__ static constexpr bool as_i(int k) { return k < 4; }
    __device__ static constexpr bool as_j(int k) { return k >= 4; }
    __device__ static constexpr bool diag(int) { return false; }
};

template <> struct W1Role<1, 1> { // diagonal part 0: (0,0) (1,0) (2,0) (3,0) (1,1)
    static constexpr int NRD = 4, NB = 5;
    __device__ static constexpr bool jreg(int) { return false; }
    __device__ static constexpr int pos(int k) { return 32 * k; }
    __device__ static constexpr int xr(int b) { return b < 4 ? b : 1; }
    __device__ static constexpr int yr(int b) { return b < 4 ? 0 : 1; }
    __device__ static constexpr int ox(int b) { return xr(b); }
    __device__ static constexpr int oy(int b) { return yr(b); }
    __device__ static constexpr bool as_i(int) { return true; }
    __device__ static constexpr bool as_j(int k) { return k < 2; }
    __device__ static constexpr bool diag(int b) { return b == 0 || b == 4; }
};

template <> struct W1Role<1, 2> { // diagonal part 1: (2,1) (3,1) (2,2) (3,2) (3,3)
    static constexpr int NRD = 3, NB = 5;  // read block k = input block k + 1
    __device__ static constexpr bool jreg(int) { return false; }
    __device__ static constexpr int pos(int k) { return 32 * (k + 1); }
    __device__ static constexpr int ox(int b) { return (b == 0 || b == 2) ? 2 : 3; }
    __device__ static constexpr int oy(int b) { return b < 2 ? 1 : (b < 4 ? 2 : 3); }
    __device__ static constexpr int xr(int b) { return ox(b) - 1; }
    __device__ static constexpr int yr(int b) { return oy(b) - 1; }
    __device__ static constexpr bool as_i(int k) { return k >= 1; }
    __device__ static constexpr bool as_j(int) { return true; }
    __device__ static constexpr bool diag(int b) { return b == 2 || b == 4; }
};

template <> struct W1Role<2, 0> { // off-diagonal tile: 64 I x 64 J
    static constexpr int NRD = 4, NB = 4;
    __device__ static constexpr bool jreg(int k) { return k >= 2; }
    __device__ static constexpr int pos(int k) { return 32 * (k & 1); }
    __device__ static constexpr int xr(int b) { return b & 1; }
    __device__ static constexpr int yr(int b) { return 2 + (b >> 1); }
    __device__ static constexpr int ox(int b) { return b & 1; }
    __device__ static constexpr int oy(int b) { return b >> 1; }
    __device__ static constexpr bool as_i(int k) { return k < 2; }
    __device__ static constexpr bool as_j(int k) { return k >= 2; }
    __device__ static constexpr bool diag(int) { return false; }
};

template <> struct W1Role<2, 1> { // diagonal tile: (0,0) (1,0) (1,1)
    static constexpr int NRD = 2, NB = 3;
    __device__ static constexpr bool jreg(int) { return false; }
    __device__ static constexpr int pos(int k) { return 32 * k; }
    __device__ static constexpr int xr(int b) { return b == 0 ? 0 : 1; }
    __device__ static constexpr int yr(int b) { return b == 2 ? 1 : 0; }
    __device__ static constexpr int ox(int b) { return xr(b); }
    __device__ static constexpr int oy(int b) { return yr(b); }
    __device__ static constexpr bool as_i(int) { return true; }
    __device__ static constexpr bool as_j(int) { return true; }
    __device__ static constexpr bool diag(int b) { return b != 1; }
};

// Wait until at most N of this wave's vector-memory operations (copies) are
// outstanding.
template <int N>
__device__ __forceinline__ void w1_wait_vm()
{
    asm volatile("s_waitcnt vmcnt(%0)" : : "n"(N) : "memory");
}

// One K step of role R: unpack the raw fragments, sum the real parts of the
// I-side rows, and issue the 4 NB MFMAs (all blocks' first product, then
// all second products, ...: the same accumulator is reused 8 (or 5) MFMAs
// later, never back to back).
template <int V, int R>
__device__ __forceinline__ void w1_kstep(const i32x2 (&Rw)[W1Role<V, R>::NRD][2],
                                         i32x16 (&accR)[W1Role<V, R>::NB],
                                         i32x16 (&accI)[W1Role<V, R>::NB],
                                         int32_t (&S)[W1Role<V, R>::NRD])
{
    typedef W1Role<V, R> Ro;
    constexpr uint32_t M = 0xF0F0F0F0u;
    i32x4 re[Ro::NRD], im[Ro::NRD], ni[Ro::NRD];
#pragma unroll
    for (int k = 0; k < Ro::NRD; ++k) {
        const u32x4 p = {(uint32_t)Rw[k][0].x, (uint32_t)Rw[k][0].y, (uint32_t)Rw[k][1].x,
                         (uint32_t)Rw[k][1].y};
        re[k] = (i32x4)(p & M);
        const u32x4 q = (p << 4) & M;
        im[k] = (i32x4)q;
        if (Ro::as_j(k)) ni[k] = (i32x4)(q ^ M);
        if (Ro::as_i(k)) {
#pragma unroll
            for (int d = 0; d < 4; ++d)
                S[k] = __builtin_amdgcn_sdot8((int)p[d], 0x10101010, S[k], false);
        }
    }
#pragma unroll
    for (int b = 0; b < Ro::NB; ++b)
        accR[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re[Ro::xr(b)], re[Ro::yr(b)], accR[b], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < Ro::NB; ++b)
        accI[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re[Ro::xr(b)], ni[Ro::yr(b)], accI[b], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < Ro::NB; ++b)
        accR[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im[Ro::xr(b)], im[Ro::yr(b)], accR[b], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < Ro::NB; ++b)
        accI[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im[Ro::xr(b)], re[Ro::yr(b)], accI[b], 0, 0, 0);
}

// V = 1: one wave per SIMD; V = 2: two.
template <int V>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(V, V)))
void xcorr_w1_kernel(W1Args a)
{
    typedef W1Geo<V> Geo;
    typedef W1Layout<V> L;
    __shared__ __attribute__((aligned(16))) uint8_t lds[Geo::NBUF * L::STAGE];

    const int lane = threadIdx.x;
    typedef __attribute__((address_space(4))) const uint32_t c_u32_t;
    typedef __attribute__((address_space(4))) const int32_t c_i32_t;
    c_u32_t *itw = (c_u32_t *)a.items;
    c_i32_t *wbeg = (c_i32_t *)a.wg_begin;
    const int it_begin = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x]);
    const int it_end = __builtin_amdgcn_readfirstlane(wbeg[blockIdx.x + 1]);
    if (it_begin >= it_end) return;
    auto item_at = [&](int it) {
        const int u = __builtin_amdgcn_readfirstlane(it);
        WgItem w;
        w.cs = itw[2 * u];
        w.ij = itw[2 * u + 1];
        return w;
    };
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds;
    constexpr uint32_t OOR = 0x80000000u;

    // Lane-derived values are recomputed where they are used from an opaque
    // copy of the lane index: hoisted out of the item loop, every role's
    // offsets would stay live beside the accumulators.
    auto fresh_lane = [&]() {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    };

    // ---- copy cursor: every stage of every item of this wave, in order,
    // then out-of-range copies (no memory traffic) for as long as asked
    int d_item = it_begin, d_stage = 0, d_nstage = 0, d_tcount = 0;
    const uint8_t *d_base = nullptr;
    uint32_t d_rowstride = 0;
    uint32_t d_voff[L::DMA];
    auto d_setup = [&](int it) {
        const int lane = fresh_lane();
        const WgItem w = item_at(it);
        const W1Sub &sb = a.subs[w.cs >> 24];
        const int f = (int)(w.cs & 0xFFFFFFu);
        const int bi = (int)(w.ij & 0xFFFu), bj = (int)((w.ij >> 12) & 0xFFFu);
        const int role = (int)(w.ij >> 24);
        const int N = sb.n_inputs;
        d_rowstride = (uint32_t)sb.n_chans * (uint32_t)N;
        d_tcount = sb.t_count;
        d_nstage = (sb.t_count + W1_TK - 1) / W1_TK;
        d_base = sb.samples + ((size_t)sb.t_begin * sb.n_chans + f) * (size_t)N;
        // unit 64 u + lane of the stage: u < IU in the I region, the rest in
        // the J region (64-byte rows: 4 units per row)
#pragma unroll
        for (int u = 0; u < L::DMA; ++u) {
            int tau, in;
            bool on;
            if (u < L::IU) {
                constexpr int UPR = Geo::IB / 16; // units per I row
                tau = (64 / UPR) * u + lane / UPR;
                const int c = w1_slot(Geo::IB, tau, lane % UPR);
                in = Geo::TILE * bi + 16 * c;
                on = in < N;
            } else {
                tau = 16 * (u - L::IU) + (lane >> 2);
                const int c = w1_slot(64, tau, lane & 3);
                in = Geo::TILE * bj + (V == 1 ? 64 * (role & 1) : 0) + 16 * c;
                on = role < 2 && in < N; // diagonal items have no J region
            }
            d_voff[u] = on ? (uint32_t)tau * d_rowstride + (uint32_t)in : OOR;
        }
    };
    int issued = 0;
    auto d_issue = [&]() {
        const bool live = d_item < it_end;
        const int t_first = d_stage * W1_TK;
        const int nt = d_tcount - t_first < W1_TK ? d_tcount - t_first : W1_TK;
        const uint64_t base = (uint64_t)(uintptr_t)(d_base + (size_t)t_first * d_rowstride);
        const i32x4 rsrc = {(int)(uint32_t)base, (int)((uint32_t)(base >> 32) & 0xFFFFu),
                            live ? (int)((uint32_t)nt * d_rowstride) : 0, 0x00020000};
        const uint32_t dst = lds_base + (uint32_t)((issued % Geo::NBUF) * L::STAGE);
#pragma unroll
        for (int u = 0; u < L::DMA; ++u) dma16(rsrc, d_voff[u], dst + (uint32_t)(u * 1024));
        ++issued;
        if (live && ++d_stage == d_nstage) {
            d_stage = 0;
            if (++d_item < it_end) d_setup(d_item);
        }
    };
    d_setup(it_begin);
#pragma unroll
    for (int k = 0; k < L::AHEAD; ++k) d_issue();

    // Make stage s (stage k of an item with tcount samples) readable: this
    // wave's copies of it have landed (AHEAD - 1 later stages may still be in
    // flight); rows past the end of the segment are cleared (their copies
    // were out of range).
    auto land = [&](int s, int k, int tcount) {
        w1_wait_vm<(L::AHEAD - 1) * L::DMA>();
        const int nt = tcount - k * W1_TK;
        if (nt < W1_TK) {
            const int lane = fresh_lane();
            uint8_t *b = lds + (s % Geo::NBUF) * L::STAGE;
#pragma unroll
            for (int u = 0; u < L::DMA; ++u) {
                const int o = 1024 * u + 16 * lane;
                const int row = o < L::JBASE ? o / Geo::IB : (o - L::JBASE) / Geo::JB;
                if (row >= nt) *(u32x4 *)(b + o) = u32x4{0u, 0u, 0u, 0u};
            }
        }
    };

    int s = 0; // global index of the stage being multiplied

    auto run = [&](auto role_c, const WgItem &w) {
        constexpr int R = decltype(role_c)::value;
        typedef W1Role<V, R> Ro;
        const int lane = fresh_lane();
        const int G = lane >> 4;
        const W1Sub &sb = a.subs[w.cs >> 24];
        const int f = (int)(w.cs & 0xFFFFFFu);
        const int bi = (int)(w.ij & 0xFFFu), bj = (int)((w.ij >> 12) & 0xFFFu);
        const int h = (int)(w.ij >> 24) & 1;
        const int tcount = sb.t_count;
        const int nst = (tcount + W1_TK - 1) / W1_TK;

        // transposing-read offsets of this role's blocks within a stage
        int fo[Ro::NRD];
#pragma unroll
        for (int k = 0; k < Ro::NRD; ++k) {
            const int pos = Ro::pos(k) + 16 * (G & 1);
            const int c = pos >> 4;
            const int m = (lane >> 1) & 7, hh = lane & 1;
            const int tau = 16 * (G >> 1) + m;
            const int rowb = Ro::jreg(k) ? Geo::JB : Geo::IB;
            fo[k] = (Ro::jreg(k) ? L::JBASE : 0) + tau * rowb + 16 * w1_slot(rowb, tau, c) + 8 * hh;
        }
        auto read = [&](int slot, i32x2 (&Rw)[Ro::NRD][2]) {
            const uint8_t *b = lds + slot * L::STAGE;
#pragma unroll
            for (int k = 0; k < Ro::NRD; ++k)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    Rw[k][i] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                        (lds_i32x2 *)(b + fo[k] + 8 * i * (Ro::jreg(k) ? Geo::JB : Geo::IB)));
        };

        i32x16 accR[Ro::NB], accI[Ro::NB];
        int32_t S[Ro::NRD];
#pragma unroll
        for (int b = 0; b < Ro::NB; ++b) {
            accR[b] = i32x16{};
            accI[b] = i32x16{};
        }
#pragma unroll
        for (int k = 0; k < Ro::NRD; ++k) S[k] = 0;

        // two fragment buffers used in turn (no copies between K steps: a
        // copy would make the compiler wait for the next stage's reads)
        i32x2 Ra[Ro::NRD][2], Rb[Ro::NRD][2];
        land(s, 0, tcount);
        read(s % Geo::NBUF, Ra);
        auto step = [&](int k, i32x2 (&Rc)[Ro::NRD][2], i32x2 (&Rn)[Ro::NRD][2]) {
            // the slot of stage s - 1 is free: its fragments were consumed by
            // the previous K step
            d_issue();
            // the reads are issued on every K step (the last one re-reads the
            // current slot, unused) so that the LDS-counter waits the
            // compiler places before the unpack count exactly these 2 NRD
            // younger reads and never wait for them
            const bool more = k + 1 < nst;
            if (more) land(s + 1, k + 1, tcount);
            read((more ? s + 1 : s) % Geo::NBUF, Rn);
            // issue them before this step's MFMAs (left alone, the scheduler
            // sinks them to the end of the chain, and the next step waits)
            __builtin_amdgcn_sched_barrier(0);
            w1_kstep<V, R>(Rc, accR, accI, S);
            ++s;
        };
        int k = 0;
        for (; k + 1 < nst; k += 2) {
            step(k, Ra, Rb);
            step(k + 1, Rb, Ra);
        }
        if (k < nst) step(k, Ra, Rb);

        // ---- flush. S: lanes l and l + 32 hold halves of the real-part sum
        // of row l % 32 of read block k.
        const int N = sb.n_inputs;
        const int r0 = Geo::TILE * bi;
        const int c0 = (V == 1 && R == 0) ? 128 * bj + 64 * h : (R == 0 ? Geo::TILE * bj : Geo::TILE * bi);
        const int r1 = r0 + Geo::TILE < N ? r0 + Geo::TILE : N;
        const int64_t tri = (int64_t)N * (N + 1) / 2;
        const int64_t rb0 = (int64_t)r0 * (r0 + 1) / 2;
        const int64_t rb1 = (int64_t)r1 * (r1 + 1) / 2;
        const size_t cell0 = (size_t)f * (size_t)tri + (size_t)rb0;
        const int nbytes = (int)((rb1 - rb0) * 8);
        const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((uint2 *)sb.dst + cell0), (short)0, nbytes, 0x00020000);
        const bool add = sb.src != nullptr;
        const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const uint2 *)(add ? sb.src : sb.dst) + cell0), (short)0, add ? nbytes : 0,
            0x00020000);
        const int lh = lane >> 5, lc = lane & 31;
        // S[k] of row l % 32 of read block k (used as I): this wave's sums
        // minus src's diagonal word of that row (src's -S_i in the raw form)
#pragma unroll
        for (int k = 0; k < Ro::NRD; ++k)
            if (Ro::as_i(k)) {
                S[k] += __shfl_xor(S[k], 32);
                int kb = 0; // output block row of read block k
#pragma unroll
                for (int b = 0; b < Ro::NB; ++b)
                    if (Ro::xr(b) == k) kb = Ro::ox(b);
                const int i = r0 + 32 * kb + lc;
                const uint32_t doff = (i < N) ? (uint32_t)((int64_t)i * (i + 1) / 2 + i - rb0) * 8u : OOR;
                const u32x2 dg = add ? __builtin_amdgcn_raw_buffer_load_b64(srs, (int)doff, 0, 0)
                                     : u32x2{0u, 0u};
                S[k] -= (int32_t)dg.y;
            }
#pragma unroll
        for (int b = 0; b < Ro::NB; ++b) {
            // the block's sums stay in accumulation registers until here, so
            // they are moved out one block at a time
            asm volatile("" : "+a"(accR[b]), "+a"(accI[b]));
#pragma unroll
            for (int e0 = 0; e0 < 16; e0 += 4) {
                // four elements at a time: keeps the scheduler from hoisting
                // every block's loads (and their registers) to the top
                __builtin_amdgcn_sched_barrier(0);
                uint32_t off[4];
                int32_t sv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = 8 * (e0 >> 2) + 4 * lh + e;
                    const int i = r0 + 32 * Ro::ox(b) + rr;
                    const int j = c0 + 32 * Ro::oy(b) + lc;
                    const int rel = (int)((int64_t)i * (i + 1) / 2 - rb0);
                    const bool ok = i < N && (!Ro::diag(b) || j <= i);
                    off[e] = ok ? (uint32_t)(rel + j) * 8u : OOR;
                    sv[e] = __shfl(S[Ro::xr(b)], rr);
                }
                u32x2 old[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    old[e] = add ? __builtin_amdgcn_raw_buffer_load_b64(srs, (int)off[e], 0, 0)
                                 : u32x2{0u, 0u};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const u32x2 v = {old[e].x + (uint32_t)(accR[b][e0 + e] >> 8),
                                     old[e].y + (uint32_t)((accI[b][e0 + e] >> 8) + sv[e])};
                    __builtin_amdgcn_raw_buffer_store_b64(v, drs, (int)off[e], 0, 0);
                }
            }
        }
        // drain the flush (its stores may complete out of order with the copies)
        dma_wait<0>();
    };

    for (int it = it_begin; it < it_end; ++it) {
        const WgItem w = item_at(it);
        const int role = (int)(w.ij >> 24);
        if constexpr (V == 1) {
            if (role < 2) run(std::integral_constant<int, 0>(), w);
            else if (role == 2) run(std::integral_constant<int, 1>(), w);
            else run(std::integral_constant<int, 2>(), w);
        } else {
            if (role < 2) run(std::integral_constant<int, 0>(), w);
            else run(std::integral_constant<int, 1>(), w);
        }
    }
    // the copies issued past the end still land in this workgroup's LDS
    dma_wait<0>();
}

} // namespace xeng
