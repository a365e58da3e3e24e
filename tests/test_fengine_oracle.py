"""Pins of the reference F-engine (oracle/fengine.py) against what the
mathematics and the library routines fix. No GPU.

* the prototype is scipy's Hamming-window FIR design of a one-channel-wide
  low-pass (an independent library routine);
* the FIR fold plus real FFT equals the modulated filter bank evaluated by
  brute force over the whole window (no fold, no FFT);
* a tone at a channel centre gives the closed-form amplitude and phase; a
  tone on a channel edge splits into two halves of -6.02 dB, as any
  windowed-sinc low-pass does at its cut-off;
* white noise gives the energy fixed by Parseval's relation;
* the requantiser rounds half to even, clips, and packs in the X-engine's
  format (decoded by the X-engine oracle's own decoder).
"""
import numpy as np
import pytest
import scipy.signal

import synth
from oracle import decode
from oracle import fengine as fe


@pytest.mark.parametrize("P,taps", [(8192, 4), (64, 4), (32, 3)])
def test_prototype_is_hamming_windowed_lowpass(P, taps):
    L = P * taps
    h = fe.prototype(P, taps)
    # firwin: ideal low-pass with cut-off 1/P of Nyquist times the window, unscaled
    ref = P * scipy.signal.firwin(L, 1.0 / P, window="hamming", scale=False)
    assert np.max(np.abs(h - ref)) < 1e-12
    w = scipy.signal.windows.hamming(L, sym=True)
    mid = L // 2 + 7
    assert h[mid] == pytest.approx(w[mid] * np.sinc((mid - (L - 1) / 2) / P), rel=1e-14)


def test_coefficients_are_18_bit_codes():
    c = fe.coefficients()
    h = fe.prototype()
    assert c.dtype == np.int64
    assert c.max() == (1 << 17) - 1 and c.min() >= -(1 << 17)
    np.testing.assert_array_equal(c, c[::-1])           # symmetric prototype
    clipped = h * 2.0 ** 17 > (1 << 17) - 0.5            # the centre taps round to 2^17
    assert 0 < clipped.sum() < 32 and np.all(c[clipped] == (1 << 17) - 1)
    err = np.abs(c * 2.0 ** -17 - h)
    assert err[~clipped].max() <= 2.0 ** -18 + 1e-15    # rounding of Q1.17 codes
    assert err[clipped].max() <= 2.0 ** -17


def brute_bank(x, m, ch, P, taps, gain):
    """Channel ch of a modulated filter bank: sum over the whole L-sample
    window, each sample weighted by the prototype and the channel's carrier."""
    c = fe.coefficients(P, taps).astype(np.float64) * 2.0 ** -17
    l = np.arange(P * taps)
    seg = x[m * P:m * P + P * taps].astype(np.float64)
    return gain / P * np.sum(c * seg * np.exp(-2j * np.pi * ch * l / P))


@pytest.mark.parametrize("P,taps", [(32, 4), (64, 3)])
def test_fold_fft_equals_modulated_bank_small(P, taps):
    x = synth.adc(11, 1, P * (taps + 3), tones=((5.0, 30.0),), n_fft=P)[0]
    for m in range(4):
        Y = fe.spectrum(x, m, 0.75, 0, P // 2, P, taps)
        ref = np.array([brute_bank(x, m, ch, P, taps, 0.75) for ch in range(P // 2)])
        np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-9 * np.max(np.abs(ref)))


def test_fold_fft_equals_modulated_bank_full_size():
    P, taps = 8192, 4
    x = synth.adc(12, 1, P * 6)[0]
    for m, chans in ((0, (0, 1, 1400, 4095)), (2, (1250, 2100, 3647))):
        Y = fe.spectrum(x, m, 1.0, 0, P // 2)
        for ch in chans:
            ref = brute_bank(x, m, ch, P, taps, 1.0)
            assert abs(Y[ch] - ref) < 1e-9 * max(1.0, abs(ref))


def tone(P, taps, f, amp, phase, n_spectra):
    s = np.arange(P * (n_spectra + taps - 1), dtype=np.float64)
    return np.rint(amp * np.cos(2 * np.pi * f * s / P + phase)).astype(np.int64)


def test_tone_at_channel_centre_closed_form():
    P, taps, c0, A, phi, gain = 8192, 4, 1400, 100.0, 0.7, 3.0
    x = tone(P, taps, c0, A, phi, 3)
    H0 = fe.prototype(P, taps).sum()
    for m in range(3):
        Y = fe.spectrum(x, m, gain, 1398, 5)
        expect = gain * A / 2.0 * np.exp(1j * phi) * H0 / P
        assert abs(Y[2] - expect) < 1e-3 * abs(expect)
        # neighbours: windowed-sinc stop band
        assert 20 * np.log10(abs(Y[1]) / abs(Y[2])) < -45
        assert 20 * np.log10(abs(Y[0]) / abs(Y[2])) < -60


def test_tone_on_channel_edge_splits_at_minus_6db():
    P, taps, c0 = 8192, 4, 2100
    x = tone(P, taps, c0 + 0.5, 100.0, 0.3, 1)
    Y = fe.spectrum(x, 0, 1.0, c0 - 1, 4)
    H0 = fe.prototype(P, taps).sum()
    full = 100.0 / 2.0 * H0 / P
    for k in (1, 2):
        assert 20 * np.log10(abs(Y[k]) / full) == pytest.approx(-6.02, abs=0.1)


def test_white_noise_energy_parseval():
    P, taps, sigma, M = 8192, 4, 16.0, 8
    x = synth.adc(13, 1, P * (M + taps - 1), sigma=sigma, tones=())[0]
    c = fe.coefficients(P, taps)
    E = np.mean([np.mean(np.abs(fe.spectrum(x, m, 1.0, 1, P // 2 - 1)) ** 2) for m in range(M)])
    # per channel: sigma^2 sum_l h[l]^2 / P^2; rounding of the samples adds 1/12
    expect = (sigma ** 2 + 1.0 / 12.0) * np.sum((c * 2.0 ** -17) ** 2) / P ** 2
    assert E == pytest.approx(expect, rel=0.02)


def test_requantise_rounding_clipping_packing():
    v = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 7.49, 7.5, 9.0, -8.5, -8.51, -20.0, 0.0, 3.2])
    Y = v + 1j * v[::-1]
    codes = fe.requantise(Y)
    re, im = decode(codes, 4)
    exp_re = np.array([0, 2, 2, 0, -2, -2, 7, 7, 7, -8, -8, -8, 0, 3])
    np.testing.assert_array_equal(re, exp_re)
    np.testing.assert_array_equal(im, exp_re[::-1])
    np.testing.assert_array_equal(codes, synth.pack4(exp_re, exp_re[::-1]))


def test_fengine_layout_and_gain():
    P, taps, N, M = 64, 4, 5, 3
    adc = synth.adc(14, N, P * (M + taps - 1), n_fft=P, tones=((10.0, 40.0),))
    codes, Y = fe.fengine(adc, M, 0.05, 3, 20, P, taps)
    assert codes.shape == (M, 20, N) and Y.shape == (M, 20, N)
    for m in range(M):
        for n in range(N):
            np.testing.assert_array_equal(Y[m, :, n], fe.spectrum(adc[n], m, 0.05, 3, 20, P, taps))
    np.testing.assert_array_equal(codes, fe.requantise(Y))
    g = fe.gain_for_rms(adc, 2.5, 3, 20, P, taps)
    _, Y2 = fe.fengine(adc[:4], 2, g, 3, 20, P, taps)
    assert np.sqrt(np.mean(np.abs(Y2) ** 2) / 2) == pytest.approx(2.5, rel=1e-9)


def test_adc_generator_law():
    x = synth.adc(15, 3, 1 << 16, tones=())
    assert x.dtype == np.int8 and x.shape == (3, 1 << 16)
    assert np.std(x.astype(np.float64)) == pytest.approx(np.sqrt(16.0 ** 2 + 1 / 12), rel=0.02)
    np.testing.assert_array_equal(x, synth.adc(15, 3, 1 << 16, tones=()))
