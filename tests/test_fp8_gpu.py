"""Parity of the FP8 (e4m3 MFMA, fp32 partial sums) engine, bit-exact.

4-bit values and their products are exact in e4m3 and fp32, and each launch
segment keeps partial sums below 2^24, so the FP8 engine must give exactly
the oracle's integers and exactly the int8 engine's output.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FP8 = 1


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rand4(rng, T, F, N, lo=-8, hi=7):
    re = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    im = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    return synth.pack4(re, im)


def run(torch, samples, engine, calls=1):
    from paper_1411_3751_amd import Correlator
    T, F, N = samples.shape
    d = torch.from_numpy(samples).cuda()
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T, in_bits=4, engine=engine)]) as c:
        for _ in range(calls):
            c.correlate([d])
        out = c.dump()[0]
        torch.cuda.synchronize()
        return out.cpu().numpy()


SHAPES16 = [(16, 3, 5), (32, 2, 64), (48, 2, 70), (96, 2, 129), (144, 2, 100), (160, 2, 33),
            (256, 3, 1000), (512, 1, 200)]


@pytest.mark.parametrize("N,F,T", SHAPES16)
def test_fp8_parity_random(torch_cuda, oracle_lib, N, F, T):
    print("case fp8 N=%d F=%d T=%d" % (N, F, T), flush=True)
    rng = np.random.default_rng(7000 + N * 10 + F + T)
    s = rand4(rng, T, F, N)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    got = run(torch_cuda, s, FP8)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "first mismatches %s" % bad[:5].tolist()


@pytest.mark.parametrize("code", [0x88, 0x77, 0x8F, 0xF8, 0x18])
def test_fp8_extremes_two_segments(torch_cuda, oracle_lib, code):
    # every sample at an extreme code for 40000 samples: one full 32768-sample
    # fp32 segment at the largest magnitudes plus a tail (with the engine's
    # offset operands u = v + 8, code 0x77 gives 450 per sample in the Re
    # partial sums: 450 * 32768 < 2^24)
    print("case fp8 extremes code=%#x" % code, flush=True)
    s = np.full((40000, 1, 32), code, np.uint8)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    assert np.array_equal(run(torch_cuda, s, FP8), want)


def test_fp8_every_code_pair(torch_cuda, oracle_lib):
    # 256 inputs, input k holds byte k at every time: all pairs of the 256
    # (re, im) codes meet in one matrix
    print("case fp8 all code pairs", flush=True)
    T = 3
    s = np.tile(np.arange(256, dtype=np.uint8)[None, None, :], (T, 1, 1))
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    assert np.array_equal(run(torch_cuda, s, FP8), want)


def test_fp8_accumulates_across_calls(torch_cuda, oracle_lib):
    print("case fp8 three calls", flush=True)
    rng = np.random.default_rng(71)
    s = rand4(rng, 300, 2, 64)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4) * 3)
    assert np.array_equal(run(torch_cuda, s, FP8, calls=3), want)


def test_fp8_and_int8_subarrays_in_one_context(torch_cuda, oracle_lib):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case mixed engines", flush=True)
    rng = np.random.default_rng(72)
    s = rand4(rng, 200, 3, 80)
    d = torch.from_numpy(s).cuda()
    subs = [dict(n_inputs=80, n_chans=3, n_time=200, engine=e) for e in (0, FP8, FP8)]
    with Correlator(subs) as c:
        c.correlate([d, d, d])
        outs = [o.cpu().numpy() for o in c.dump()]
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    for o in outs:
        assert np.array_equal(o, want)
