"""Pins of the CPU oracle against what the mathematics fixes.

Nothing here uses the GPU library. Each test pins the oracle to something
other than itself: brute force through numpy's complex matrix product, a
hand-worked example, closed forms (rank-1 signals, autocorrelations),
invariances of the definition, and the encoder in ``synth`` (an independent
implementation of the 4+4-bit format).
"""
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def cplx(re, im):
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def brute(re, im):
    """numpy: X X^H per channel on complex128 (exact for these integer sizes)."""
    x = cplx(re, im)  # [T][F][N]
    xt = np.transpose(x, (1, 2, 0))  # [F][N][T]
    return xt @ np.conj(np.transpose(xt, (0, 2, 1)))


def tri_of(full):
    n = full.shape[-1]
    ii, jj = np.tril_indices(n)
    out = np.stack([full[..., ii, jj].real, full[..., ii, jj].imag], axis=-1)
    return out.astype(np.int64)


def rand_nibbles(rng, shape, lo=-8, hi=7):
    return (rng.integers(lo, hi + 1, size=shape).astype(np.int8),
            rng.integers(lo, hi + 1, size=shape).astype(np.int8))


@pytest.mark.parametrize("N,F,T", [(1, 1, 1), (3, 2, 5), (17, 3, 64), (32, 2, 129), (64, 1, 33)])
def test_brute_force_4bit(oracle_lib, N, F, T):
    rng = np.random.default_rng(1000 + N * 7 + T)
    re, im = rand_nibbles(rng, (T, F, N))
    v = oracle_lib.correlate(synth.pack4(re, im), 4)
    assert np.array_equal(v, tri_of(brute(re, im)))


@pytest.mark.parametrize("N,F,T", [(1, 1, 3), (5, 2, 7), (40, 2, 50)])
def test_brute_force_8bit(oracle_lib, N, F, T):
    rng = np.random.default_rng(2000 + N)
    re, im = rand_nibbles(rng, (T, F, N), -127, 127)
    v = oracle_lib.correlate(synth.pack8(re, im), 8)
    assert np.array_equal(v, tri_of(brute(re, im)))


def test_every_nibble_code_roundtrip(oracle_lib):
    # synth.pack4 and the oracle's decoder are independent implementations of
    # the byte format; all 256 (re, im) pairs must survive the round trip.
    r, i = np.meshgrid(np.arange(-8, 8), np.arange(-8, 8), indexing="ij")
    b = synth.pack4(r.astype(np.int8), i.astype(np.int8))
    assert sorted(b.ravel().tolist()) == list(range(256))
    dr, di = oracle_lib.decode(b.reshape(1, 1, -1), 4)
    assert np.array_equal(dr.ravel(), r.ravel()) and np.array_equal(di.ravel(), i.ravel())


@pytest.mark.parametrize("byte,re,im", [(0x10, 1, 0), (0x01, 0, 1), (0x80, -8, 0), (0x08, 0, -8),
                                        (0xFF, -1, -1), (0x7F, 7, -1), (0x88, -8, -8), (0x77, 7, 7)])
def test_nibble_order(oracle_lib, byte, re, im):
    # real part in bits 7..4, imaginary in bits 3..0; autocorrelation at T=1 is |x|^2
    s = np.array([[[byte]]], np.uint8)
    v = oracle_lib.correlate(s, 4)
    assert v[0, 0, 0] == re * re + im * im and v[0, 0, 1] == 0
    dr, di = oracle_lib.decode(s, 4)
    assert dr.item() == re and di.item() == im


def test_worked_example(oracle_lib):
    with open(os.path.join(HERE, "golden", "worked_example.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    N, F, T = map(int, rows[0])
    data = np.array([int(x, 16) for x in rows[1]], np.uint8).reshape(T, F, N)
    want = np.array([[int(a), int(b)] for a, b in rows[2:]], np.int64).reshape(F, N * (N + 1) // 2, 2)
    assert np.array_equal(oracle_lib.correlate(data, 4), want)


def test_conjugation_convention_rank1(oracle_lib):
    # x_i(t) = g_i q(t)  =>  V_ij = g_i conj(g_j) sum_t |q(t)|^2 (closed form)
    rng = np.random.default_rng(7)
    gains = np.array([1, 1j, -1, -1j, 1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j, 0, 1], np.complex128)
    N, T = len(gains), 300
    q = rng.integers(-3, 4, size=T) + 1j * rng.integers(-3, 4, size=T)
    x = gains[None, :] * q[:, None]  # [T][N]
    re = x.real.astype(np.int8)[:, None, :]
    im = x.imag.astype(np.int8)[:, None, :]
    v = oracle_lib.correlate(synth.pack4(re, im), 4)[0]
    p = float(np.sum(np.abs(q) ** 2))
    full = np.outer(gains, np.conj(gains)) * p
    assert np.array_equal(v, tri_of(full[None])[0])
    # x_1 = i x_0 => V_10 = i |q|^2: the imaginary part is +p, fixing conj on the second index
    assert v[1 * 2 // 2 + 0, 0] == 0 and v[1, 1] == p


def test_closure_phase_rank1(oracle_lib):
    # a single point source (rank-1 data) has zero closure phase: Im(V_ij V_jk V_ki) = 0
    rng = np.random.default_rng(11)
    gains = np.array([1, 1j, -1 + 1j, 1 - 1j, -1, 2, -2j], np.complex128)
    T = 200
    q = rng.integers(-3, 4, size=T) + 1j * rng.integers(-3, 4, size=T)
    x = gains[None, :] * q[:, None]
    v = oracle_lib.correlate(synth.pack4(x.real.astype(np.int8)[:, None, :],
                                         x.imag.astype(np.int8)[:, None, :]), 4)
    full = np.round(oracle_lib.unpack_tri(v, len(gains))[0]).astype(np.complex128)
    n = len(gains)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                c = full[i, j] * full[j, k] * full[k, i]
                assert c.imag == 0


def test_autocorrelations(oracle_lib):
    rng = np.random.default_rng(3)
    re, im = rand_nibbles(rng, (77, 4, 9))
    v = oracle_lib.correlate(synth.pack4(re, im), 4)
    power = (re.astype(np.int64) ** 2 + im.astype(np.int64) ** 2).sum(axis=0)  # [F][N]
    for i in range(9):
        k = i * (i + 1) // 2 + i
        assert np.array_equal(v[:, k, 0], power[:, i])
        assert np.all(v[:, k, 1] == 0)
        assert np.all(v[:, k, 0] >= 0)


def test_time_additivity(oracle_lib):
    rng = np.random.default_rng(5)
    re, im = rand_nibbles(rng, (100, 3, 12))
    s = synth.pack4(re, im)
    whole = oracle_lib.correlate(s, 4)
    acc = np.zeros_like(whole)
    oracle_lib.accumulate(acc, np.ascontiguousarray(s[:37]), 4)
    oracle_lib.accumulate(acc, np.ascontiguousarray(s[37:]), 4)
    assert np.array_equal(acc, whole)


def test_covariances(oracle_lib):
    rng = np.random.default_rng(9)
    N, T = 10, 90
    re, im = rand_nibbles(rng, (T, 2, N), -7, 7)
    base = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(re, im), 4), N)
    # input permutation permutes V
    perm = rng.permutation(N)
    vp = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(re[:, :, perm], im[:, :, perm]), 4), N)
    assert np.array_equal(vp, base[:, perm][:, :, perm])
    # x -> conj(x) gives conj(V)
    vc = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(re, -im), 4), N)
    assert np.array_equal(vc, np.conj(base))
    # x -> -x and x -> i x leave V unchanged
    vn = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(-re, -im), 4), N)
    vi = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(-im, re), 4), N)
    assert np.array_equal(vn, base) and np.array_equal(vi, base)
    # time order does not matter
    tp = rng.permutation(T)
    vt = oracle_lib.unpack_tri(oracle_lib.correlate(synth.pack4(re[tp], im[tp]), 4), N)
    assert np.array_equal(vt, base)


def test_special_cases(oracle_lib):
    # all-zero input gives zero
    z = np.zeros((13, 2, 5), np.uint8)
    assert not oracle_lib.correlate(z, 4).any()
    # every sample -8-8i: V_ij = (-8-8i)(-8+8i) T = 128 T
    T = 31
    s = np.full((T, 1, 6), 0x88, np.uint8)
    v = oracle_lib.correlate(s, 4)
    assert np.all(v[..., 0] == 128 * T) and np.all(v[..., 1] == 0)
    # T = 1: the outer product x x^H
    x = np.array([2 - 3j, -8 + 7j, 0 + 1j])
    s1 = synth.pack4(x.real.astype(np.int8)[None, None, :], x.imag.astype(np.int8)[None, None, :])
    v1 = oracle_lib.correlate(s1, 4)[0]
    assert np.array_equal(v1, tri_of(np.outer(x, np.conj(x))[None])[0])


def test_channel_selection_matches_full(oracle_lib):
    rng = np.random.default_rng(13)
    re, im = rand_nibbles(rng, (40, 9, 7))
    s = synth.pack4(re, im)
    full = oracle_lib.correlate(s, 4)
    sel = [8, 0, 4]
    assert np.array_equal(oracle_lib.correlate(s, 4, chans=sel), full[sel])


def test_narrow_detects_overflow(oracle_lib):
    ok = np.array([[2**31 - 1, -2**31]], np.int64)
    assert np.array_equal(oracle_lib.narrow(ok), ok.astype(np.int32))
    with pytest.raises(OverflowError):
        oracle_lib.narrow(np.array([2**31], np.int64))


def test_projection_check_accepts_and_rejects(oracle_lib):
    rng = np.random.default_rng(17)
    N = 24
    re, im = rand_nibbles(rng, (60, 3, N))
    s = synth.pack4(re, im)
    vis = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    w = rng.integers(-4, 5, size=(N, 2)).astype(np.int64)
    for f in range(3):
        assert oracle_lib.projection_check(s, 4, f, vis[f], w) == 0
    bad = vis[1].copy()
    bad[17, 1] += 1  # one planted error in one imaginary part
    assert oracle_lib.projection_check(s, 4, 1, bad, w) > 0
    bad = vis[2].copy()
    bad[0, 0] -= 1  # an autocorrelation off by one
    assert oracle_lib.projection_check(s, 4, 2, bad, w) > 0


def test_tone_lands_in_its_channels(oracle_lib):
    # statistical sanity of the generator + definition, not parity: the common
    # tone (amplitude 1.5) shows as Re V_ij / T ~ |A|^2 = 2.25 for i != j only in
    # the tone channels
    s, re, im, meta = synth.workload("leda_gulp", n_inputs=8, n_chans=16, n_time=4096,
                                     components=True)
    v = oracle_lib.correlate(s, 4)
    cross = [i * (i + 1) // 2 + j for i in range(8) for j in range(i)]
    mean = v[:, cross, 0].mean(axis=1) / meta["n_time"]
    tones = synth.tone_channels(16)
    assert tones == [2, 6, 10, 14]
    for f in range(16):
        if f in tones:
            assert 1.6 < mean[f] < 2.9
        else:
            assert abs(mean[f]) < 0.5


def test_generator_histogram():
    # the 4-bit draw follows the clipped, rounded Gaussian pmf (sigma 2.5)
    from math import erf, sqrt
    _, re, im, _ = synth.workload("tiny", components=True)
    counts = np.bincount(re.ravel().astype(np.int64) + 8, minlength=16)
    n = re.size
    cdf = lambda z: 0.5 * (1 + erf(z / (2.5 * sqrt(2))))
    for k, c in enumerate(counts):
        v = k - 8
        lo = -np.inf if v == -8 else v - 0.5
        hi = np.inf if v == 7 else v + 0.5
        p = (1.0 if hi == np.inf else cdf(hi)) - (0.0 if lo == -np.inf else cdf(lo))
        sd = np.sqrt(n * p * (1 - p))
        assert abs(c - n * p) < 6 * sd + 5
