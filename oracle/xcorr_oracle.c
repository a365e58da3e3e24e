/*
 * X-engine oracle: the plain CPU definition of the correlator's output.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header, table or constant with
 * the GPU library.
 *
 * What it computes (Section 2, Fig. 2 caption: the X-engines cross-multiply
 * and time-average the channelised signals one antenna pair at a time;
 * Section 2.5: spectra are read in groups, cross-multiplied and averaged, and
 * groups are summed to the dump cadence):
 *
 *   for every channel f, input i, input j <= i:
 *     V[f][i][j] = sum_t x_i(t, f) * conj(x_j(t, f))
 *     Re V = sum_t (xr_i xr_j + xi_i xi_j)
 *     Im V = sum_t (xi_i xr_j - xr_i xi_j)
 *
 * summed exactly in int64. "Averaged" is read as a plain sum (the caller knows
 * the sample count). The lower triangle i >= j, autocorrelations included, is
 * stored at the packed index i(i+1)/2 + j as an (re, im) pair. Inputs are the
 * paper's 4+4-bit complex samples (Section 2.2: requantisation to 4+4 bits),
 * one byte each with the real part in the high nibble, or the 8+8-bit form the
 * CPU layer promotes them to (Section 2.4), two int8 per sample.
 *
 * The loops are the definition written out: no blocking, no reordering beyond
 * gathering one channel's samples into per-input rows first.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Two's-complement value of a 4-bit field (Section 2.2: 4+4-bit samples).
 * The range is [-8, 7]; -8 is a legal code. */
static int nibble_value(unsigned v)
{
    return v >= 8 ? (int)v - 16 : (int)v;
}

/* Decode sample idx of a stream (Section 2.2 / Section 2.4 formats). */
static void decode(const void *samples, int in_bits, size_t idx, int *re, int *im)
{
    if (in_bits == 4) {
        unsigned b = ((const uint8_t *)samples)[idx];
        *re = nibble_value(b >> 4);
        *im = nibble_value(b & 15u);
    } else {
        const int8_t *s = (const int8_t *)samples;
        *re = s[2 * idx];
        *im = s[2 * idx + 1];
    }
}

int oracle_decode(const void *samples, int in_bits, int64_t count, int32_t *re, int32_t *im)
{
    if (!samples || !re || !im || count < 0 || (in_bits != 4 && in_bits != 8))
        return -1;
    for (int64_t k = 0; k < count; k++) {
        int r, i;
        decode(samples, in_bits, (size_t)k, &r, &i);
        re[k] = r;
        im[k] = i;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * acc[c][k][2] += visibility sums of channel chans[c] (or channel c when chans
 * is NULL, n_sel = n_chans) over the n_time samples of a [T][F][N] stream.
 * acc is caller-owned int64 [n_sel][N(N+1)/2][2]. Running sums across calls
 * give the integration over groups (Section 2.5). Returns 0, or -1 on bad
 * arguments.
 */
int oracle_accumulate(const void *samples, int in_bits, int64_t n_time, int n_chans,
                      int n_inputs, const int32_t *chans, int n_sel, int64_t *acc)
{
    if (!samples || !acc || n_time < 0 || n_chans <= 0 || n_inputs <= 0 ||
        (in_bits != 4 && in_bits != 8))
        return -1;
    if (!chans)
        n_sel = n_chans;
    for (int c = 0; c < n_sel; c++)
        if (chans && (chans[c] < 0 || chans[c] >= n_chans))
            return -1;
    const int64_t N = n_inputs, T = n_time;
    const int64_t tri = N * (N + 1) / 2;
    int bad = 0;

#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_sel; c++) {
        const int64_t f = chans ? chans[c] : c;
        /* gather channel f into per-input rows: xr[i][t], xi[i][t] */
        int32_t *xr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * T + 1));
        int32_t *xi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * T + 1));
        if (!xr || !xi) {
            free(xr);
            free(xi);
#pragma omp atomic write
            bad = 1;
            continue;
        }
        for (int64_t t = 0; t < T; t++)
            for (int64_t i = 0; i < N; i++) {
                int r, im;
                decode(samples, in_bits, (size_t)((t * n_chans + f) * N + i), &r, &im);
                xr[i * T + t] = r;
                xi[i * T + t] = im;
            }
        int64_t *out = acc + (size_t)c * (size_t)tri * 2;
        for (int64_t i = 0; i < N; i++) {
            for (int64_t j = 0; j <= i; j++) {
                int64_t re = 0, im = 0;
                const int32_t *ar = xr + i * T, *ai = xi + i * T;
                const int32_t *br = xr + j * T, *bi = xi + j * T;
                for (int64_t t = 0; t < T; t++) {
                    /* x_i * conj(x_j) */
                    re += (int64_t)ar[t] * br[t] + (int64_t)ai[t] * bi[t];
                    im += (int64_t)ai[t] * br[t] - (int64_t)ar[t] * bi[t];
                }
                const int64_t k = i * (i + 1) / 2 + j;
                out[2 * k] += re;
                out[2 * k + 1] += im;
            }
        }
        free(xr);
        free(xi);
    }
    return bad ? -2 : 0;
}

/*
 * Narrow int64 sums to the int32 output words. Returns the number of values
 * outside [INT32_MIN, INT32_MAX] (those are written saturated); 0 means the
 * output is exact.
 */
int64_t oracle_narrow(const int64_t *acc, int32_t *out, int64_t count)
{
    int64_t over = 0;
    for (int64_t k = 0; k < count; k++) {
        int64_t v = acc[k];
        if (v > INT32_MAX) {
            out[k] = INT32_MAX;
            over++;
        } else if (v < INT32_MIN) {
            out[k] = INT32_MIN;
            over++;
        } else {
            out[k] = (int32_t)v;
        }
    }
    return over;
}

/*
 * Projection check of one channel's dump (for dumps too large for the full
 * definition). With V the full Hermitian matrix rebuilt from the stored lower
 * triangle (V[j][i] = conj(V[i][j])), the definition gives, for any complex
 * vector w,
 *     V w = sum_t x(t) (x(t)^H w),
 * which costs O(N T) instead of O(N^2 T). w holds small complex integers
 * (int64 [N][2]); everything is exact in int64.
 * vis: int32 [N(N+1)/2][2] lower triangle of channel f, summed over the
 * n_time samples of this stream. Returns the number of mismatching rows of
 * V w (0 = consistent), or -1 on bad arguments.
 */
int64_t oracle_projection_check(const void *samples, int in_bits, int64_t n_time, int n_chans,
                                int n_inputs, int chan, const int32_t *vis, const int64_t *w)
{
    if (!samples || !vis || !w || n_time < 0 || chan < 0 || chan >= n_chans || n_inputs <= 0)
        return -1;
    const int64_t N = n_inputs;
    int64_t *lhs = (int64_t *)calloc((size_t)(2 * N), sizeof(int64_t));
    int64_t *rhs = (int64_t *)calloc((size_t)(2 * N), sizeof(int64_t));
    int32_t *xr = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *xi = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!lhs || !rhs || !xr || !xi) {
        free(lhs); free(rhs); free(xr); free(xi);
        return -1;
    }
    /* lhs = V w */
    for (int64_t i = 0; i < N; i++) {
        for (int64_t j = 0; j < N; j++) {
            int64_t vr, vi;
            if (j <= i) {
                const int64_t k = i * (i + 1) / 2 + j;
                vr = vis[2 * k];
                vi = vis[2 * k + 1];
            } else {
                const int64_t k = j * (j + 1) / 2 + i;
                vr = vis[2 * k];
                vi = -(int64_t)vis[2 * k + 1];
            }
            lhs[2 * i] += vr * w[2 * j] - vi * w[2 * j + 1];
            lhs[2 * i + 1] += vr * w[2 * j + 1] + vi * w[2 * j];
        }
    }
    /* rhs = sum_t x(t) * (x(t)^H w) */
    for (int64_t t = 0; t < n_time; t++) {
        int64_t sr = 0, si = 0; /* s = sum_j conj(x_j) w_j */
        for (int64_t j = 0; j < N; j++) {
            int r, im;
            decode(samples, in_bits, (size_t)((t * n_chans + chan) * N + j), &r, &im);
            xr[j] = r;
            xi[j] = im;
            sr += (int64_t)r * w[2 * j] + (int64_t)im * w[2 * j + 1];
            si += (int64_t)r * w[2 * j + 1] - (int64_t)im * w[2 * j];
        }
        for (int64_t i = 0; i < N; i++) {
            rhs[2 * i] += (int64_t)xr[i] * sr - (int64_t)xi[i] * si;
            rhs[2 * i + 1] += (int64_t)xr[i] * si + (int64_t)xi[i] * sr;
        }
    }
    int64_t bad = 0;
    for (int64_t i = 0; i < N; i++)
        if (lhs[2 * i] != rhs[2 * i] || lhs[2 * i + 1] != rhs[2 * i + 1])
            bad++;
    free(lhs); free(rhs); free(xr); free(xi);
    return bad;
}
