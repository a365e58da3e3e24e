"""Reference F-engine: polyphase filter bank, FFT, requantisation to 4+4 bits.

Test infrastructure only: nothing in the product path imports this module.
It states in plain numpy (fp64 for the FFT, exact integers for the FIR) what
the library's GPU F-engine computes, following Section 2.2:

* a 4-tap, 8192-point PFB, made of an FIR filter followed by an FFT; the
  filter is a Hamming-windowed prototype with 18-bit coefficients;
* the FFT's 18+18-bit path divides by 2 at each internal stage, which over the
  log2(8192) radix-2 stages scales the transform by 1/8192;
* one average digital gain over the band, then requantisation to 4+4-bit
  complex samples;
* a contiguous group of channels is selected (2398 channels, 30-88 MHz, in the
  paper's system) and written for the X-engine in [time][channel][input] order.

Readings where the paper is silent (each listed in the design notes):

* prototype: h[l] = w[l] sinc((l - (L-1)/2) / P), l < L = taps P, with the
  symmetric Hamming window w[l] = 0.54 - 0.46 cos(2 pi l / (L - 1)), i.e. a
  windowed ideal low-pass one channel wide;
* 18-bit coefficients: c[l] = clip(rint(2^17 h[l]), -2^17, 2^17 - 1), the
  signed Q1.17 code of h, so that h is recovered as c 2^-17;
* the FIR of spectrum m weights the L samples starting at m P in time order
  and folds them: y_m[k] = sum_tap c[tap P + k] x[(m + tap) P + k], k < P;
* Y_m[ch] = gain 2^-17 / P * sum_k y_m[k] exp(-2 pi i k ch / P);
* requantisation rounds half to even (rint) and clips each component to
  [-8, 7]; the byte is re << 4 | im in two's complement nibbles, the
  X-engine's input format.
"""
from __future__ import annotations

import numpy as np

P_FFT = 8192
TAPS = 4
COEF_BITS = 18


def prototype(P: int = P_FFT, taps: int = TAPS) -> np.ndarray:
    """fp64 Hamming-windowed sinc prototype h[l], l < taps P (Section 2.2)."""
    L = taps * P
    l = np.arange(L, dtype=np.float64)
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * l / (L - 1))
    return w * np.sinc((l - (L - 1) / 2.0) / P)


def coefficients(P: int = P_FFT, taps: int = TAPS) -> np.ndarray:
    """18-bit signed FIR coefficients c[l] (int64), h = c 2^-17."""
    lim = 1 << (COEF_BITS - 1)
    return np.clip(np.rint(prototype(P, taps) * lim), -lim, lim - 1).astype(np.int64)


def fir(x: np.ndarray, m: int, P: int = P_FFT, taps: int = TAPS, c=None) -> np.ndarray:
    """Exact integer FIR output y_m[k], k < P, of one input's samples ``x``
    (int), for spectrum m: samples [m P, (m + taps) P)."""
    c = coefficients(P, taps) if c is None else c
    seg = np.asarray(x[m * P:(m + taps) * P], np.int64)
    if seg.size != taps * P:
        raise ValueError("spectrum %d needs samples up to %d" % (m, (m + taps) * P))
    return (c * seg).reshape(taps, P).sum(axis=0)


def spectrum(x: np.ndarray, m: int, gain: float, chan0: int, n_chans: int, P: int = P_FFT,
             taps: int = TAPS, c=None) -> np.ndarray:
    """Gain-scaled channel values Y_m[chan0 .. chan0 + n_chans) (complex128):
    the FIR output through a P-point real DFT (numpy's rfft in fp64), scaled
    by gain 2^-17 / P."""
    y = fir(x, m, P, taps, c).astype(np.float64)
    Y = np.fft.rfft(y)
    return Y[chan0:chan0 + n_chans] * (gain * 2.0 ** -(COEF_BITS - 1) / P)


def requantise(Y: np.ndarray) -> np.ndarray:
    """4+4-bit codes of complex values: rint each component, clip to [-8, 7],
    pack re in bits 7..4 and im in bits 3..0."""
    re = np.clip(np.rint(Y.real), -8, 7).astype(np.int64)
    im = np.clip(np.rint(Y.imag), -8, 7).astype(np.int64)
    return (((re & 15) << 4) | (im & 15)).astype(np.uint8)


def fengine(adc: np.ndarray, n_spectra: int, gain: float, chan0: int, n_chans: int,
            P: int = P_FFT, taps: int = TAPS, spectra=None):
    """F-engine of ``adc`` (int8 [N][S]) for spectra m < n_spectra (or the
    listed ``spectra``). Returns (codes uint8 [M][n_chans][N], Y complex128
    [M][n_chans][N]), the X-engine's [time][channel][input] layout."""
    N = adc.shape[0]
    ms = list(range(n_spectra)) if spectra is None else list(spectra)
    c = coefficients(P, taps)
    Y = np.empty((len(ms), n_chans, N), np.complex128)
    for a, m in enumerate(ms):
        for n in range(N):
            Y[a, :, n] = spectrum(adc[n], m, gain, chan0, n_chans, P, taps, c)
    return requantise(Y), Y


def gain_for_rms(adc: np.ndarray, target: float, chan0: int, n_chans: int, P: int = P_FFT,
                 taps: int = TAPS, n_spectra: int = 2) -> float:
    """The one band-average gain that brings the rms of each component of the
    selected channels to ``target`` (measured on the first spectra of the
    first inputs); the paper applies one such factor across the band."""
    _, Y = fengine(adc[:min(4, adc.shape[0])], n_spectra, 1.0, chan0, n_chans, P, taps)
    rms = np.sqrt(np.mean(Y.real ** 2 + Y.imag ** 2) / 2.0)
    return float(target / rms)
