/*
 * Counter-based quantised-Gaussian sample generator (host side).
 *
 * Input generation only: nothing here correlates anything. The same
 * definition is implemented for the GPU in synth/gpu_gen.hip; both draw
 * element (t, f, i, component) of a stream from a counter, so any slice of a
 * stream (a time range, a subset of channels) is reproducible on its own.
 *
 * Definition (identical on both sides):
 *   key  = mix(seed)
 *   c    = ((t * F + f) * N + i) * 2 + comp        t: absolute sample index,
 *                                                  comp 0 = real, 1 = imag
 *   u    = mix(key + (c + 1) * 0x9E3779B97F4A7C15) >> 32
 *   v    = lo + #{ k in [0, L - 1) : u >= thr[k] }  L = hi - lo + 1 levels
 * where mix is the SplitMix64 output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014; the
 * 0xBF58476D1CE4E5B9 / 0x94D049BB133111EB variant) and thr[k] =
 * floor(2^32 Phi((lo + k + 1/2 - a) / sigma)) are computed by the caller
 * (a = tone component at time t, 0 without tone). Since u is uniform on
 * [0, 2^32), v has the law of clip(round(sigma g + a), lo, hi), g ~ N(0, 1).
 *
 * Output: 4-bit streams as one byte per sample, ((re & 15) << 4) | (im & 15);
 * 8-bit streams as int8 (re, im) pairs. Optionally the int8 components too.
 */
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline int level(uint32_t u, const uint32_t *thr, int n_thr)
{
    /* number of thresholds <= u (thresholds are non-decreasing) */
    int lo = 0, hi = n_thr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u >= thr[mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/*
 * Fill samples of times [t0, t0 + n_time) for the channels chans[0..n_sel)
 * (all channels if chans is NULL; then n_sel must equal n_chans).
 *   out       4-bit: uint8 [n_time][n_sel][n_inputs]; 8-bit: int8 [...][2]
 *   re, im    optional int8 [n_time][n_sel][n_inputs] components (may be NULL)
 *   thr_base  [n_lv - 1] thresholds without tone
 *   thr_tone  [n_time][2][n_lv - 1] thresholds with the tone at each time
 *             (re, im), used for channels with tone_chan[f] != 0; may be NULL
 */
void synth_fill(void *out, int8_t *re, int8_t *im, int in_bits, int64_t n_time, int64_t t0,
                int32_t n_chans, int32_t n_inputs, const int32_t *chans, int32_t n_sel,
                uint64_t seed, int32_t lo, int32_t n_lv, const uint32_t *thr_base,
                const uint32_t *thr_tone, const uint8_t *tone_chan, int threads)
{
    const uint64_t key = mix64(seed);
    const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
    const int n_thr = n_lv - 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t t = 0; t < n_time; ++t)
        for (int32_t s = 0; s < n_sel; ++s) {
            const int32_t f = chans ? chans[s] : s;
            const int tone = thr_tone && tone_chan && tone_chan[f];
            const uint32_t *tr = tone ? thr_tone + (size_t)t * 2 * n_thr : thr_base;
            const uint32_t *ti = tone ? tr + n_thr : thr_base;
            const uint64_t c0 = (((uint64_t)(t0 + t) * (uint64_t)n_chans + (uint64_t)f) *
                                 (uint64_t)n_inputs) * 2u;
            const size_t o = ((size_t)t * (size_t)n_sel + (size_t)s) * (size_t)n_inputs;
            for (int32_t i = 0; i < n_inputs; ++i) {
                const uint64_t c = c0 + 2u * (uint64_t)i;
                const uint32_t ur = (uint32_t)(mix64(key + (c + 1u) * gamma) >> 32);
                const uint32_t ui = (uint32_t)(mix64(key + (c + 2u) * gamma) >> 32);
                const int vr = lo + level(ur, tr, n_thr);
                const int vi = lo + level(ui, ti, n_thr);
                if (in_bits == 4)
                    ((uint8_t *)out)[o + i] = (uint8_t)(((vr & 15) << 4) | (vi & 15));
                else {
                    ((int8_t *)out)[2 * (o + i)] = (int8_t)vr;
                    ((int8_t *)out)[2 * (o + i) + 1] = (int8_t)vi;
                }
                if (re) re[o + i] = (int8_t)vr;
                if (im) im[o + i] = (int8_t)vi;
            }
        }
}
