"""GPU F-engine (PFB + FFT + 4+4-bit requantisation) against the reference
F-engine in oracle/fengine.py.

Floating-point tolerance. The FIR is exact on both sides (integers); the GPU
then converts y (|y| < 2^26) to fp32 and runs a 4096-point complex FFT in three
radix-16 passes plus the real-FFT split, all in fp32 with fp32 twiddles. The
rounding error of such an FFT grows with log2 of its length; per element it
stays far below TOL_K u log2(P) rms(Y), u = 2^-24, with rms(Y) the rms over all
channels of that spectrum (the error spreads evenly over the channels), and
TOL_K = 32 leaves a margin of three or more over the largest error seen.

4+4-bit codes are compared exactly wherever the reference value lies farther
than that tolerance from a rounding boundary (k + 1/2); within it, either
neighbouring code is accepted.
"""
import numpy as np
import pytest

import synth
from oracle import fengine as fe

pytestmark = pytest.mark.gpu

P = fe.P_FFT
TAPS = fe.TAPS
TOL_K = 32.0
U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(torch, adc, n_spectra, chan0, n_chans, gain, stride_pad=0, with_spec=True):
    from paper_1411_3751_amd import FEngine
    N, S = adc.shape
    stride = S + stride_pad
    host = np.zeros((N, stride), np.int8)
    host[:, :S] = adc
    d_adc = torch.from_numpy(host).cuda()
    out = torch.empty((n_spectra, n_chans, N), dtype=torch.uint8, device="cuda")
    spec = torch.empty((n_spectra, n_chans, N), dtype=torch.complex64, device="cuda") if with_spec else None
    with FEngine(N, chan0, n_chans, gain) as f:
        f.run(d_adc, n_spectra, out, spec)
        torch.cuda.synchronize()
        group = f.group
    return out.cpu().numpy(), (spec.cpu().numpy() if with_spec else None), group


def tolerance(adc_row, m, gain):
    Yall = fe.spectrum(adc_row, m, gain, 0, P // 2 + 1)
    rms = np.sqrt(np.mean(np.abs(Yall) ** 2))
    return TOL_K * U * np.log2(P) * rms


def check(codes, spec, ref_codes, ref_Y, tol):
    """tol: [M][N] per (spectrum, input). Spectra within tol; codes exact away
    from rounding boundaries, else one of the two neighbours."""
    t = tol[:, None, :]
    if spec is not None:
        err = np.abs(spec.astype(np.complex128) - ref_Y)
        print("max err/tol %.3g" % np.max(err / t), flush=True)
        assert np.all(err <= t), "max err/tol %.3g" % np.max(err / t)
    near = np.zeros(ref_Y.shape, bool)
    for comp in (ref_Y.real, ref_Y.imag):
        frac = np.abs(comp - np.floor(comp) - 0.5)
        near |= (frac <= t) & (comp > -8.5 - t) & (comp < 7.5 + t)
    far = ~near
    np.testing.assert_array_equal(codes[far], ref_codes[far])
    if near.any():
        tn = np.broadcast_to(t, ref_Y.shape)[near]
        lo = fe.requantise(ref_Y[near] - (1 + 1j) * tn)
        hi = fe.requantise(ref_Y[near] + (1 + 1j) * tn)
        got = codes[near]
        for part in (lambda c: c >> 4, lambda c: c & 15):
            g, a, b = (part(v.astype(np.int32)) for v in (got, lo, hi))
            sx = lambda v: np.where(v >= 8, v - 16, v)
            assert np.all((sx(g) >= sx(a)) & (sx(g) <= sx(b)))
    return int(near.sum())


CASES = [
    # (seed, N, n_spectra, chan0, n_chans, stride_pad): groups 4, 2, 1, ragged channel counts
    (1, 16, 4, 1250, 300, 0),
    (2, 24, 3, 1000, 1500, 8),
    (3, 12, 2, 0, 4096, 0),
    (4, 6, 2, 4000, 96, 16),
    (5, 7, 3, 1399, 5, 0),
    (6, 1, 1, 4095, 1, 0),
]


@pytest.mark.parametrize("seed,N,M,chan0,F,pad", CASES)
def test_fengine_matches_reference(torch_cuda, seed, N, M, chan0, F, pad):
    print("case fengine seed=%d N=%d M=%d chan0=%d F=%d pad=%d" % (seed, N, M, chan0, F, pad),
          flush=True)
    adc = synth.adc(100 + seed, N, P * (M + TAPS - 1))
    gain = fe.gain_for_rms(adc, 2.5, 1250, 2398, n_spectra=min(2, M))
    codes, spec, group = run_gpu(torch_cuda, adc, M, chan0, F, gain, pad)
    assert group == max(g for g in (1, 2, 4) if N % g == 0)
    ref_codes, ref_Y = fe.fengine(adc, M, gain, chan0, F)
    tol = np.array([[tolerance(adc[n], m, gain) for n in range(N)] for m in range(M)])
    near = check(codes, spec, ref_codes, ref_Y, tol)
    assert near <= max(2, codes.size // 1000)
    # codes alone (no spectrum output) are the same
    codes2, _, _ = run_gpu(torch_cuda, adc, M, chan0, F, gain, pad, with_spec=False)
    np.testing.assert_array_equal(codes2, codes)


def test_fengine_full_size_sampled(torch_cuda):
    """The benchmark's shape (512 inputs, channels 1250..3647, 64 spectra per
    call): sampled (spectrum, input) pairs against the reference."""
    torch = torch_cuda
    from paper_1411_3751_amd import FEngine
    N, M, chan0, F = 512, 64, 1250, 2398
    S = P * (M + TAPS - 1)
    print("case fengine full N=%d M=%d F=%d" % (N, M, F), flush=True)
    d_adc = synth.adc_device(7, N, S, "cuda")
    rows = [0, 1, 63, 64, 255, 300, 510, 511]
    host_rows = d_adc[rows].cpu().numpy()
    gain = fe.gain_for_rms(host_rows, 2.5, chan0, F)
    out = torch.empty((M, F, N), dtype=torch.uint8, device="cuda")
    spec = torch.empty((M, F, N), dtype=torch.complex64, device="cuda")
    with FEngine(N, chan0, F, gain) as f:
        assert f.group == 4
        f.run(d_adc, M, out, spec)
        torch.cuda.synchronize()
    ms = [0, 1, 31, 62, 63]
    codes = out.cpu().numpy()[ms][:, :, rows]
    Y = spec.cpu().numpy()[ms][:, :, rows]
    ref_codes, ref_Y = fe.fengine(host_rows, 0, gain, chan0, F, spectra=ms)
    tol = np.array([[tolerance(host_rows[a], m, gain) for a in range(len(rows))] for m in ms])
    check(codes, Y, ref_codes, ref_Y, tol)


def test_fengine_maximum_inputs(torch_cuda):
    """The largest input count the boundary takes (65535, odd: one input per
    workgroup), one spectrum, sampled inputs against the reference."""
    torch = torch_cuda
    from paper_1411_3751_amd import FEngine
    N, M, chan0, F = 65535, 1, 1392, 24
    print("case fengine max inputs N=%d" % N, flush=True)
    d_adc = synth.adc_device(9, N, P * TAPS, "cuda")
    rows = [0, 1, 4097, 32767, 65533, 65534]
    host_rows = d_adc[rows].cpu().numpy()
    gain = fe.gain_for_rms(host_rows, 2.5, 1250, 2398, n_spectra=1)
    out = torch.empty((M, F, N), dtype=torch.uint8, device="cuda")
    spec = torch.empty((M, F, N), dtype=torch.complex64, device="cuda")
    with FEngine(N, chan0, F, gain) as f:
        assert f.group == 1
        f.run(d_adc, M, out, spec)
        torch.cuda.synchronize()
    codes = out.cpu().numpy()[:, :, rows]
    Y = spec.cpu().numpy()[:, :, rows]
    ref_codes, ref_Y = fe.fengine(host_rows, M, gain, chan0, F)
    tol = np.array([[tolerance(host_rows[a], 0, gain) for a in range(len(rows))]])
    check(codes, Y, ref_codes, ref_Y, tol)
    del d_adc


def test_fengine_feeds_xengine(torch_cuda):
    """F-engine output straight into the X-engine; against the reference
    F-engine's codes correlated by the reference X-engine."""
    torch = torch_cuda
    from oracle import correlate, narrow
    from paper_1411_3751_amd import Correlator, FEngine
    N, M, chan0, F = 16, 8, 1390, 16
    adc = synth.adc(32, N, P * (M + TAPS - 1))   # a seed with no value within tol of a boundary
    gain = fe.gain_for_rms(adc, 2.5, 1250, 2398)
    ref_codes, ref_Y = fe.fengine(adc, M, gain, chan0, F)
    tol = np.array([[tolerance(adc[n], m, gain) for n in range(N)] for m in range(M)])
    for comp in (ref_Y.real, ref_Y.imag):
        frac = np.abs(comp - np.floor(comp) - 0.5)
        assert np.all(frac > tol[:, None, :]), "seed has a value at a rounding boundary"
    d_adc = torch.from_numpy(adc).cuda()
    codes = torch.empty((M, F, N), dtype=torch.uint8, device="cuda")
    with FEngine(N, chan0, F, gain) as f:
        f.run(d_adc, M, codes)
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=M, in_bits=4)]) as xc:
        xc.correlate([codes])
        got = xc.dump()[0].cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(codes.cpu().numpy(), ref_codes)
    np.testing.assert_array_equal(got, narrow(correlate(ref_codes, 4)))


def test_fengine_into_stream_ring(torch_cuda):
    """The FX pipeline: the F-engine writes each gulp straight into the X-engine
    ring slot on the ring's ingest stream (raw-pointer call). The ring's dump
    must equal the X-engine run on the same F-engine output produced by
    ordinary calls. The two components are each checked against their
    references above; this checks their composition through the ring."""
    torch = torch_cuda
    from paper_1411_3751_amd import Correlator, FEngine, Stream
    N, M, chan0, F, G = 16, 64, 1380, 24, 2          # gulp = 64 spectra, dump after 2 gulps
    S = P * (G * M + TAPS - 1)
    adc = synth.adc(41, N, S)
    d_adc = torch.from_numpy(adc).cuda()
    gain = fe.gain_for_rms(adc, 2.5, 1250, 2398)
    codes = torch.empty((G * M, F, N), dtype=torch.uint8, device="cuda")
    hd = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, pin_memory=True)]
    with FEngine(N, chan0, F, gain) as f:
        f.run(d_adc, G * M, codes)
        torch.cuda.synchronize()
        with Stream(dict(n_inputs=N, n_chans=F, n_time=M), n_slots=2, dump_every=G, host_dumps=hd) as st:
            for g in range(G):
                ptr, ist = st.next_slot()
                f.run_ptr(d_adc.data_ptr() + g * M * P, S, M, ptr, 0, ist)
                st.push()
            st.dump_wait(0)
            got = hd[0].numpy().copy()
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=G * M)]) as xc:
        xc.correlate([codes])
        want = xc.dump()[0].cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got, want)


def test_fengine_errors(torch_cuda):
    torch = torch_cuda
    from paper_1411_3751_amd import FEngine, XengError
    with pytest.raises(XengError):
        FEngine(8, 4000, 200, 1.0)            # channels past 4096
    with pytest.raises(XengError):
        FEngine(8, 0, 16, 0.0)                # gain
    with pytest.raises(XengError):
        FEngine(0, 0, 16, 1.0)                # inputs
    with FEngine(8, 0, 16, 1.0) as f:
        out = torch.empty((2, 16, 8), dtype=torch.uint8, device="cuda")
        short = torch.zeros((8, P * 4), dtype=torch.int8, device="cuda")   # needs 5 P for 2 spectra
        with pytest.raises(XengError):
            f.run(short, 2, out)
        odd = torch.zeros((8, P * 5 + 4), dtype=torch.int8, device="cuda")  # stride not a multiple of 8
        with pytest.raises(XengError):
            f.run(odd, 2, out)
        with pytest.raises(ValueError):
            f.run(torch.zeros((7, P * 5), dtype=torch.int8, device="cuda"), 2, out)
        torch.cuda.synchronize()
