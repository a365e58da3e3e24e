"""Quantised-Gaussian voltage streams shaped like the LEDA-512 F-engine output.

The paper's F-engine requantises channelised voltages to 4+4-bit complex
samples after one band-average digital gain (Section 2.2); its test plan adds
continuous-wave tones (Section 5). The sky data itself is not available, so
these generators stand in for it:

* every real and imaginary component is ``clip(rint(sigma * g + a), lo, hi)``
  with ``g ~ N(0, 1)`` (numpy ``rint``: round half to even) and ``a`` the tone
  component where a tone is present, else 0;
* 4-bit streams use ``[lo, hi] = [-8, 7]``; 8-bit streams ``[-127, 127]``;
* the common tone is ``s(t) = A exp(i 2 pi (nu t + phi0))``, identical on all
  inputs, in the channels ``(2m+1) F / 8`` for ``m = 0..3``.

Layout of a stream is ``[time][channel][input]`` (post corner turn, Fig. 2).
Draws are made per block of ``BLOCK_T`` time samples with a generator seeded
by ``(seed, block index)``, so the result does not depend on how many blocks
are drawn at once or in which thread.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED_BASE = 14113751
BLOCK_T = 64


def tone_channels(n_chans: int) -> list[int]:
    """Channels that carry the injected tone: (2m+1)F/8 for m = 0..3."""
    if n_chans < 8:
        return []
    return sorted({(2 * m + 1) * n_chans // 8 for m in range(4)})


def tone_series(t0: int, n_t: int, amp: float, nu: float, phi0: float = 0.0):
    """Complex tone amplitude a(t) = amp * exp(i 2 pi (nu t + phi0)) for t in [t0, t0+n_t)."""
    t = np.arange(t0, t0 + n_t, dtype=np.float64)
    ph = 2.0 * np.pi * (nu * t + phi0)
    return amp * np.cos(ph), amp * np.sin(ph)


def _draw_block(seed: int, blk: int, n_t: int, n_chans: int, n_inputs: int,
                sigma: float, lo: int, hi: int, tone):
    rng = np.random.default_rng([seed, blk])
    shape = (n_t, n_chans, n_inputs)
    re = rng.standard_normal(shape, dtype=np.float32)
    im = rng.standard_normal(shape, dtype=np.float32)
    re *= np.float32(sigma)
    im *= np.float32(sigma)
    if tone is not None:
        amp, nu, phi0, chans = tone
        if chans:
            tr, ti = tone_series(blk * BLOCK_T, n_t, amp, nu, phi0)
            cs = np.asarray(chans)
            re[:, cs, :] += tr.astype(np.float32)[:, None, None]
            im[:, cs, :] += ti.astype(np.float32)[:, None, None]
    np.rint(re, out=re)
    np.rint(im, out=im)
    np.clip(re, lo, hi, out=re)
    np.clip(im, lo, hi, out=im)
    return re.astype(np.int8), im.astype(np.int8)


def draw_stream(seed: int, n_time: int, n_chans: int, n_inputs: int, sigma: float,
                lo: int = -8, hi: int = 7, tone=None, threads: int | None = None):
    """Integer components (re, im), each int8 ``[n_time][n_chans][n_inputs]``.

    ``tone`` is ``(amp, nu, phi0, channels)`` or ``None``.
    """
    re = np.empty((n_time, n_chans, n_inputs), np.int8)
    im = np.empty_like(re)
    n_blk = (n_time + BLOCK_T - 1) // BLOCK_T

    def work(b):
        t0 = b * BLOCK_T
        n_t = min(BLOCK_T, n_time - t0)
        r, i = _draw_block(seed, b, n_t, n_chans, n_inputs, sigma, lo, hi, tone)
        re[t0:t0 + n_t] = r
        im[t0:t0 + n_t] = i

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if n_blk == 1 or threads == 1:
        for b in range(n_blk):
            work(b)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(n_blk)))
    return re, im


def pack4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """One byte per complex sample: real part in bits 7..4, imaginary in 3..0,
    both two's complement, each in [-8, 7]."""
    re = np.asarray(re)
    im = np.asarray(im)
    if re.size and (re.min() < -8 or re.max() > 7 or im.min() < -8 or im.max() > 7):
        raise ValueError("4-bit components must lie in [-8, 7]")
    b = ((re.astype(np.int16) & 0xF) << 4) | (im.astype(np.int16) & 0xF)
    return np.ascontiguousarray(b.astype(np.uint8))


def pack8(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Two bytes per complex sample, int8 (re, im) interleaved: [..., 2]."""
    return np.ascontiguousarray(np.stack([np.asarray(re, np.int8), np.asarray(im, np.int8)], axis=-1))


# Workload recipes. Sizes follow the paper's 512-input system (Table 1) and the
# configurations the benchmark and parity tests use.
WORKLOADS = {
    "tiny": dict(n_inputs=32, n_chans=16, n_time=1024, sigma=2.5, in_bits=4, tone=False, k=0),
    "leda_gulp": dict(n_inputs=512, n_chans=128, n_time=8192, sigma=2.5, in_bits=4, tone=True, k=1),
    "fp8_variant": dict(n_inputs=512, n_chans=256, n_time=16384, sigma=2.5, in_bits=4, tone=False, k=2),
    "int8_variant": dict(n_inputs=512, n_chans=256, n_time=16384, sigma=20.0, in_bits=8, tone=False, k=2),
}
TONE_AMP = 1.5
TONE_NU = 1.0 / 128.0


def workload(name: str, subarray: int = 0, n_time: int | None = None,
             n_chans: int | None = None, n_inputs: int | None = None):
    """Draw a named workload; returns ``(samples, re, im, meta)``.

    ``samples`` is the packed device format (uint8 ``[T][F][N]`` for 4-bit,
    int8 ``[T][F][N][2]`` for 8-bit). Sizes can be overridden to draw a smaller
    instance with the same recipe.
    """
    w = dict(WORKLOADS[name])
    T = n_time or w["n_time"]
    F = n_chans or w["n_chans"]
    N = n_inputs or w["n_inputs"]
    seed = SEED_BASE + w["k"] + 100 * subarray
    if w["in_bits"] == 4:
        lo, hi = -8, 7
    else:
        lo, hi = -127, 127
    tone = (TONE_AMP, TONE_NU, 0.0, tone_channels(F)) if w["tone"] else None
    re, im = draw_stream(seed, T, F, N, w["sigma"], lo, hi, tone)
    samples = pack4(re, im) if w["in_bits"] == 4 else pack8(re, im)
    meta = dict(w, n_time=T, n_chans=F, n_inputs=N, seed=seed)
    return samples, re, im, meta
