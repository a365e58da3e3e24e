"""The allocation-free correlate-and-dump (xeng_correlate_dump_static),
called through the C ABI, against the context path (xeng_correlate_dump) on
the same inputs: bit-exact on two calls in a row, the second on a smaller
input, for 4-bit input on the int8 and FP8 engines and 8-bit input."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rand(rng, T, F, N, in_bits):
    lo, hi = (-8, 7) if in_bits == 4 else (-128, 127)
    re = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    im = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    return synth.pack4(re, im) if in_bits == 4 else synth.pack8(re, im)


def static_call(torch, x, sub):
    from paper_1411_3751_amd import xeng
    lib = xeng.load()
    N, F = sub["n_inputs"], sub["n_chans"]
    d = torch.from_numpy(x).cuda()
    out = torch.full((F, N * (N + 1) // 2, 2), -1, dtype=torch.int32, device="cuda")
    s = xeng.Subarray(N, F, sub["n_time"], sub.get("in_bits", 4), sub.get("engine", 0))
    rc = lib.xeng_correlate_dump_static(ctypes.byref(s), ctypes.c_void_p(d.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.xeng_last_error().decode()
    torch.cuda.synchronize()
    return out.cpu().numpy()


def context_call(torch, x, sub):
    from paper_1411_3751_amd import Correlator
    with Correlator([sub]) as c:
        out = c.correlate_dump([torch.from_numpy(x).cuda()])[0]
        torch.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("in_bits,engine", [(4, 0), (4, 1), (8, 0)])
def test_static_matches_context_twice(torch_cuda, oracle_lib, in_bits, engine):
    rng = np.random.default_rng(61 + in_bits + engine)
    shapes = [(512, 16, 4096), (144, 3, 300)] if in_bits == 4 else [(264, 8, 2048), (40, 3, 300)]
    for (N, F, T) in shapes:
        print("case static N=%d F=%d T=%d in_bits=%d engine=%d" % (N, F, T, in_bits, engine),
              flush=True)
        sub = dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits, engine=engine)
        x = rand(rng, T, F, N, in_bits)
        got = static_call(torch_cuda, x, sub)
        want = context_call(torch_cuda, x, sub)
        bad = np.argwhere(got != want)
        assert bad.size == 0, "first mismatches %s" % bad[:5].tolist()
    # the smaller call also against the oracle
    assert np.array_equal(got, oracle_lib.narrow(oracle_lib.correlate(x, in_bits)))


def test_static_limits(torch_cuda):
    from paper_1411_3751_amd import xeng
    lib = xeng.load()
    torch = torch_cuda
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    o = torch.zeros(16, dtype=torch.int32, device="cuda")
    for sub in [xeng.Subarray(20, 1, 64, 4, 0),        # N not a multiple of 16
                xeng.Subarray(16, 1, 40000, 4, 0),     # more than one launch segment
                xeng.Subarray(65520, 5, 8, 4, 0)]:     # more tiles than the static list holds
        rc = lib.xeng_correlate_dump_static(ctypes.byref(sub), ctypes.c_void_p(d.data_ptr()),
                                            ctypes.c_void_p(o.data_ptr()), None)
        assert rc == xeng.XENG_EINVAL, lib.xeng_last_error().decode()
