"""Quantised-Gaussian voltage streams shaped like the LEDA-512 F-engine output.

The paper's F-engine requantises channelised voltages to 4+4-bit complex
samples after one band-average digital gain (Section 2.2); its test plan adds
continuous-wave tones (Section 5). The sky data itself is not available, so
these generators stand in for it:

* every real and imaginary component has the law of
  ``clip(round(sigma * g + a), lo, hi)`` with ``g ~ N(0, 1)`` and ``a`` the
  tone component where a tone is present, else 0;
* 4-bit streams use ``[lo, hi] = [-8, 7]``; 8-bit streams ``[-127, 127]``;
* the common tone is ``s(t) = A exp(i phi(t))``, identical on all inputs, in
  the channels ``(2m+1) F / 8`` for ``m = 0..3``; ``phi(t) = 2 pi (nu t +
  phi0)`` for a fixed tone, or a phase-continuous drift across gulps.

Each component is drawn from a counter (stream seed, absolute time, channel,
input, re/im) through the SplitMix64 output function and a table of uint32
thresholds (``csynth.c`` states the definition; ``gpu_gen.hip`` implements the
same one on the GPU), so any time range or channel subset of a stream can be
regenerated on its own, bit for bit, on the host or on the device.

Layout of a stream is ``[time][channel][input]`` (post corner turn, Fig. 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsynth.so")
SRC = os.path.join(HERE, "csynth.c")

SEED_BASE = 14113751
TONE_AMP = 1.5
TONE_NU = 1.0 / 128.0

_lib = None


def build(force: bool = False) -> str:
    """Compile the host generator (gcc, OpenMP) next to its source."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_fill.restype = None
        lib.synth_fill.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def tone_channels(n_chans: int) -> list[int]:
    """Channels that carry the injected tone: (2m+1)F/8 for m = 0..3."""
    if n_chans < 8:
        return []
    return sorted({(2 * m + 1) * n_chans // 8 for m in range(4)})


def tone_series(t0: int, n_t: int, amp: float, nu: float, phi0: float = 0.0):
    """Tone components amp * (cos, sin)(2 pi (nu t + phi0)) for t in [t0, t0+n_t)."""
    t = np.arange(t0, t0 + n_t, dtype=np.float64)
    ph = 2.0 * np.pi * (nu * t + phi0)
    return amp * np.cos(ph), amp * np.sin(ph)


def drift_phase(t: np.ndarray, gulp: int, nu0: float = TONE_NU, dnu: float = 1e-5):
    """Phase (radians) of a tone whose frequency steps by dnu per gulp of
    ``gulp`` samples (nu_g = nu0 + g dnu), continuous across gulps."""
    t = np.asarray(t, np.int64)
    g = t // gulp
    # phase at the start of gulp g: 2 pi gulp sum_{h<g} nu_h
    start = 2.0 * np.pi * gulp * (nu0 * g + dnu * g * (g - 1) / 2.0)
    return start + 2.0 * np.pi * (nu0 + dnu * g) * (t - g * gulp)


def thresholds(lo: int, hi: int, sigma: float, a=0.0) -> np.ndarray:
    """uint32 thresholds floor(2^32 Phi((lo + k + 1/2 - a) / sigma)), k < hi - lo.

    ``a`` may be an array (one table per entry): the result then has shape
    ``a.shape + (hi - lo,)``.
    """
    from scipy.special import ndtr
    a = np.asarray(a, np.float64)
    b = lo + np.arange(hi - lo, dtype=np.float64) + 0.5
    z = (b - a[..., None]) / sigma
    th = np.floor(ndtr(z) * 4294967296.0)
    return np.clip(th, 0, 4294967295).astype(np.uint32)


def stream(seed: int, n_time: int, n_chans: int, n_inputs: int, in_bits: int, sigma: float,
           t0: int = 0, chans=None, tone=None, components: bool = False, threads: int = 0):
    """Draw times [t0, t0 + n_time) of a stream for channels ``chans`` (all if None).

    ``tone`` is ``(amp, phase_fn, tone_chans)`` with ``phase_fn(t)`` the phase
    in radians at absolute times t, or None. Returns ``(samples, re, im)``:
    samples uint8 ``[T][S][N]`` (4-bit) or int8 ``[T][S][N][2]`` (8-bit); re, im
    int8 ``[T][S][N]`` when ``components`` else None.
    """
    lo, hi = (-8, 7) if in_bits == 4 else (-127, 127)
    n_lv = hi - lo + 1
    sel = np.arange(n_chans, dtype=np.int32) if chans is None else np.asarray(chans, np.int32)
    n_sel = int(sel.size)
    if in_bits == 4:
        out = np.empty((n_time, n_sel, n_inputs), np.uint8)
    else:
        out = np.empty((n_time, n_sel, n_inputs, 2), np.int8)
    re = np.empty((n_time, n_sel, n_inputs), np.int8) if components else None
    im = np.empty((n_time, n_sel, n_inputs), np.int8) if components else None
    base = thresholds(lo, hi, sigma)
    thr_tone = None
    tone_mask = None
    if tone is not None and tone[2]:
        amp, phase_fn, tchans = tone
        ph = phase_fn(np.arange(t0, t0 + n_time, dtype=np.int64))
        a = np.stack([amp * np.cos(ph), amp * np.sin(ph)], axis=1)  # [T][2]
        thr_tone = np.ascontiguousarray(thresholds(lo, hi, sigma, a))  # [T][2][L-1]
        tone_mask = np.zeros(n_chans, np.uint8)
        tone_mask[list(tchans)] = 1
    lib = _load()
    ptr = lambda x: None if x is None else x.ctypes.data
    lib.synth_fill(ptr(out), ptr(re), ptr(im), in_bits, n_time, t0, n_chans, n_inputs,
                   ptr(sel), n_sel, ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), lo, n_lv,
                   ptr(base), ptr(thr_tone), ptr(tone_mask), int(threads))
    return out, re, im


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
    # subarray s of the batch takes (n_inputs, n_chans) = BATCH_SHAPES[s]
    "batch": dict(n_inputs=None, n_chans=None, n_time=4096, sigma=2.5, in_bits=4, tone=False, k=3),
    # the batch's first subarray on its own (same seed): the small-N, memory-bound shape
    "n64": dict(n_inputs=64, n_chans=512, n_time=4096, sigma=2.5, in_bits=4, tone=False, k=3),
}
# Batched subarrays of uneven size: (N, F) with equal input bytes per call for N >= 256.
BATCH_SHAPES = [(64, 512), (256, 256), (512, 128), (1024, 64), (2048, 32)]


def fixed_tone(n_chans: int, amp: float = TONE_AMP, nu: float = TONE_NU, phi0: float = 0.0):
    """The workloads' tone: amp exp(i 2 pi (nu t + phi0)) in tone_channels(F)."""
    return (amp, lambda t: 2.0 * np.pi * (nu * np.asarray(t, np.float64) + phi0),
            tone_channels(n_chans))


def workload(name: str, subarray: int = 0, n_time: int | None = None,
             n_chans: int | None = None, n_inputs: int | None = None, chans=None,
             components: bool = False):
    """Draw a named workload; returns ``(samples, re, im, meta)``.

    ``samples`` is the packed device format (uint8 ``[T][F][N]`` for 4-bit,
    int8 ``[T][F][N][2]`` for 8-bit), restricted to ``chans`` if given. Sizes
    can be overridden to draw a smaller instance with the same recipe. ``re``
    and ``im`` are the int8 components when ``components`` is true, else None.
    """
    w = dict(WORKLOADS[name])
    if name == "batch":
        w["n_inputs"], w["n_chans"] = BATCH_SHAPES[subarray]
    T = n_time or w["n_time"]
    F = n_chans or w["n_chans"]
    N = n_inputs or w["n_inputs"]
    seed = SEED_BASE + w["k"] + 100 * subarray
    tone = fixed_tone(F) if w["tone"] else None
    samples, re, im = stream(seed, T, F, N, w["in_bits"], w["sigma"], chans=chans, tone=tone,
                             components=components)
    meta = dict(w, n_time=T, n_chans=F, n_inputs=N, seed=seed)
    return samples, re, im, meta


PACKET_MAGIC = 0x4C454441  # "LEDA", the packet header's magic word


def packet_stride(pkt_time: int, pkt_chans: int, pkt_inputs: int, in_bits: int = 4) -> int:
    payload = pkt_time * pkt_chans * pkt_inputs * (in_bits // 4)
    return 16 + (payload + 15) // 16 * 16


def packetize(samples: np.ndarray, t0: int, pkt_time: int, pkt_chans: int, pkt_inputs: int,
              in_bits: int = 4) -> np.ndarray:
    """Cut a stream slice [T][F][N](x2) starting at absolute time t0 into
    F-engine packets (16-byte header: uint64 t0, uint16 chan0, uint16 input0,
    uint32 magic; payload [pkt_time][pkt_chans][pkt_inputs] samples), in
    (time block, channel block, input block) order. Returns uint8
    [n_packets][stride]."""
    s = np.ascontiguousarray(samples).view(np.uint8)
    T, F, N = samples.shape[:3]
    bps = in_bits // 4
    s = s.reshape(T, F, N * bps)
    nt, nf, ni = T // pkt_time, F // pkt_chans, N // pkt_inputs
    if nt * pkt_time != T or nf * pkt_chans != F or ni * pkt_inputs != N:
        raise ValueError("packet blocks must divide the stream slice")
    stride = packet_stride(pkt_time, pkt_chans, pkt_inputs, in_bits)
    out = np.zeros((nt, nf, ni, stride), np.uint8)
    blk = s.reshape(nt, pkt_time, nf, pkt_chans, ni, pkt_inputs * bps).transpose(0, 2, 4, 1, 3, 5)
    payload = pkt_time * pkt_chans * pkt_inputs * bps
    out[..., 16:16 + payload] = blk.reshape(nt, nf, ni, payload)
    hdr = np.zeros((nt, nf, ni, 2), np.uint64)
    tb, fb, ib = np.meshgrid(np.arange(nt), np.arange(nf), np.arange(ni), indexing="ij")
    hdr[..., 0] = (t0 + tb * pkt_time).astype(np.uint64)
    hdr[..., 1] = ((fb * pkt_chans).astype(np.uint64) | ((ib * pkt_inputs).astype(np.uint64) << 16)
                   | (np.uint64(PACKET_MAGIC) << np.uint64(32)))
    out[..., :16] = hdr.view(np.uint8).reshape(nt, nf, ni, 16)
    return out.reshape(nt * nf * ni, stride)


# F-engine input: real 8-bit ADC samples (Section 2.2: an 8-bit, 16-input ADC
# clocked at 196.608 MHz feeds the PFB). Gaussian receiver noise plus
# continuous-wave tones, the test signal the paper injects into an assembled
# F-engine (Section 5). Frequencies are in channel units (cycles per sample
# times the FFT length), so a tone at 1400.0 sits at the centre of channel 1400.
ADC_SIGMA = 16.0
ADC_FFT = 8192
ADC_TONES = ((1400.0, 40.0), (2100.25, 24.0), (3000.5, 12.0), (3600.0, 90.0))


def adc(seed: int, n_inputs: int, n_samples: int, sigma: float = ADC_SIGMA, tones=ADC_TONES,
        n_fft: int = ADC_FFT) -> np.ndarray:
    """int8 ``[n_inputs][n_samples]`` ADC samples: round(sigma g + sum_k A_k
    cos(2 pi f_k s / n_fft + phi_kn)), clipped to [-128, 127]; g ~ N(0, 1) from
    numpy's PCG64 seeded with ``seed``; phase phi_kn = 2 pi (0.37 n + 0.11 k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = sigma * rng.standard_normal((n_inputs, n_samples))
    s = np.arange(n_samples, dtype=np.float64)
    for k, (f, amp) in enumerate(tones or ()):
        ph = 2.0 * np.pi * (0.37 * np.arange(n_inputs) + 0.11 * k)
        x += amp * np.cos(2.0 * np.pi * f * s[None, :] / n_fft + ph[:, None])
    return np.clip(np.rint(x), -128, 127).astype(np.int8)


def adc_device(seed: int, n_inputs: int, n_samples: int, device, sigma: float = ADC_SIGMA,
               tones=ADC_TONES, n_fft: int = ADC_FFT):
    """The same recipe as :func:`adc` drawn on a torch device (torch's own
    generator, so the values differ from :func:`adc`; the law is the same).
    Built one input row block at a time to bound the float32 temporaries."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((n_inputs, n_samples), dtype=torch.int8, device=device)
    s = torch.arange(n_samples, dtype=torch.float64, device=device)
    step = max(1, (1 << 26) // max(1, n_samples))
    for n0 in range(0, n_inputs, step):
        n1 = min(n_inputs, n0 + step)
        x = sigma * torch.randn((n1 - n0, n_samples), generator=g, device=device)
        for k, (f, amp) in enumerate(tones or ()):
            ph = 2.0 * np.pi * (0.37 * torch.arange(n0, n1, device=device, dtype=torch.float64) + 0.11 * k)
            cyc = torch.remainder(f * s / n_fft, 1.0)
            x += (amp * torch.cos(2.0 * np.pi * cyc[None, :] + ph[:, None])).float()
        out[n0:n1] = torch.clamp(torch.round(x), -128, 127).to(torch.int8)
    return out
