"""The input generator follows its stated counter-based definition.

A pure-Python restatement of the definition (SplitMix64 output function on a
per-element counter, then a threshold count) is compared with the compiled
generator on scattered elements, and slices of a stream drawn separately
must equal the same slices of the whole stream.
"""
import numpy as np

import synth

M64 = (1 << 64) - 1


def mix64(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def element(seed, t, f, i, comp, F, N, thr, lo):
    key = mix64(seed & M64)
    c = ((t * F + f) * N + i) * 2 + comp
    u = mix64((key + (c + 1) * 0x9E3779B97F4A7C15) & M64) >> 32
    return lo + int(np.sum(u >= thr.astype(np.int64)))


def test_definition_4bit_and_8bit():
    rng = np.random.default_rng(1)
    for in_bits, lo, hi, sigma in [(4, -8, 7, 2.5), (8, -127, 127, 20.0)]:
        T, F, N, t0, seed = 40, 5, 37, 1000, 123456789
        s, re, im = synth.stream(seed, T, F, N, in_bits, sigma, t0=t0, components=True)
        thr = synth.thresholds(lo, hi, sigma)
        for _ in range(200):
            t, f, i = int(rng.integers(T)), int(rng.integers(F)), int(rng.integers(N))
            assert re[t, f, i] == element(seed, t0 + t, f, i, 0, F, N, thr, lo)
            assert im[t, f, i] == element(seed, t0 + t, f, i, 1, F, N, thr, lo)
        if in_bits == 4:
            assert np.array_equal(s, synth.pack4(re, im))
        else:
            assert np.array_equal(s, synth.pack8(re, im))


def test_tone_thresholds_follow_the_phase():
    T, F, N = 64, 8, 4
    tone = synth.fixed_tone(F)
    s, re, im = synth.stream(9, T, F, N, 4, 2.5, tone=tone, components=True)
    thr = synth.thresholds(-8, 7, 2.5, np.stack([1.5 * np.cos(2 * np.pi * np.arange(T) / 128),
                                                 1.5 * np.sin(2 * np.pi * np.arange(T) / 128)], 1))
    for t, f, i in [(0, 1, 0), (5, 3, 2), (63, 5, 3), (17, 7, 1)]:
        assert re[t, f, i] == element(9, t, f, i, 0, F, N, thr[t, 0], -8)
        assert im[t, f, i] == element(9, t, f, i, 1, F, N, thr[t, 1], -8)
    # a channel without tone uses the plain table
    plain = synth.thresholds(-8, 7, 2.5)
    assert re[3, 0, 1] == element(9, 3, 0, 1, 0, F, N, plain, -8)


def test_slices_are_independent():
    whole, _, _ = synth.stream(77, 300, 6, 20, 4, 2.5, tone=synth.fixed_tone(6))
    part, _, _ = synth.stream(77, 100, 6, 20, 4, 2.5, t0=150, chans=[4, 1],
                              tone=synth.fixed_tone(6))
    assert np.array_equal(part, whole[150:250][:, [4, 1]])


def test_drift_phase_is_continuous():
    g = 8192
    t = np.arange(3 * g)
    ph = synth.drift_phase(t, g)
    d = np.diff(ph)
    # step inside gulp h is 2 pi nu_h; at a boundary it is the previous gulp's
    nu = synth.TONE_NU + 1e-5 * (t[:-1] // g)
    assert np.allclose(d, 2 * np.pi * nu, rtol=0, atol=1e-9)
