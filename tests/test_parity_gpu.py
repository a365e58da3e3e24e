"""Parity of the HIP X-engine with the CPU oracle (bit-exact), through the C ABI.

Every case prints its shape before running so that a failure names it.
"""
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


def rand_stream(rng, T, F, N, in_bits, lo=None, hi=None):
    if in_bits == 4:
        lo = -8 if lo is None else lo
        hi = 7 if hi is None else hi
        re = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
        im = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
        return synth.pack4(re, im)
    lo = -128 if lo is None else lo
    hi = 127 if hi is None else hi
    re = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    im = rng.integers(lo, hi + 1, size=(T, F, N)).astype(np.int8)
    return synth.pack8(re, im)


def gpu_once(torch, samples, in_bits, engine=0):
    from paper_1411_3751_amd import Correlator
    T, F, N = samples.shape[:3]
    d = torch.from_numpy(samples).cuda()
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits, engine=engine)]) as c:
        c.correlate([d])
        out = c.dump()[0]
        torch.cuda.synchronize()
        return out.cpu().numpy()


SHAPES = [
    # (N, F, T): tile variants (N <= 32, <= 64, > 64), ragged N and T, several tiles
    (1, 2, 1), (2, 3, 7), (5, 2, 63), (31, 3, 64), (32, 2, 65), (33, 2, 100),
    (64, 2, 129), (65, 2, 64), (100, 3, 200), (128, 2, 256), (130, 2, 77),
    (200, 2, 300), (257, 1, 130), (384, 1, 64),
    # multiples of 16 (direct LDS staging for 4-bit): tails, partial tiles, diagonal tiles
    (16, 3, 5), (48, 2, 70), (96, 2, 64), (144, 2, 100), (160, 2, 33), (256, 3, 1000),
    (512, 1, 200),
]


@pytest.mark.parametrize("in_bits", [4, 8])
@pytest.mark.parametrize("N,F,T", SHAPES)
def test_parity_random(torch_cuda, oracle_lib, N, F, T, in_bits):
    print("case N=%d F=%d T=%d in_bits=%d" % (N, F, T, in_bits), flush=True)
    rng = np.random.default_rng(N * 1000 + F * 10 + T + in_bits)
    s = rand_stream(rng, T, F, N, in_bits)
    want = oracle_lib.narrow(oracle_lib.correlate(s, in_bits))
    got = gpu_once(torch_cuda, s, in_bits)
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, "first mismatches %s" % bad[:5].tolist()


@pytest.mark.parametrize("in_bits,code", [(4, 0x88), (4, 0x77), (4, 0x8F), (8, -128), (8, 127)])
def test_extreme_values(torch_cuda, oracle_lib, in_bits, code):
    # saturated inputs (all -8-8i, 7+7i, ...) exercise the largest products
    print("case extremes in_bits=%d code=%d" % (in_bits, code), flush=True)
    T, F, N = 300, 2, 70
    if in_bits == 4:
        s = np.full((T, F, N), code, np.uint8)
    else:
        s = np.full((T, F, N, 2), code, np.int8)
    want = oracle_lib.narrow(oracle_lib.correlate(s, in_bits))
    assert np.array_equal(gpu_once(torch_cuda, s, in_bits), want)


def test_tiny_workload(torch_cuda, oracle_lib):
    # N=32 inputs, 16 channels, 1024 samples, quantised Gaussian (sigma 2.5)
    s, _, _, _ = synth.workload("tiny")
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    assert np.array_equal(gpu_once(torch_cuda, s, 4), want)


def test_multi_segment_call(torch_cuda, oracle_lib):
    # a call longer than one launch segment (32768 samples) is split and summed
    print("case multi-segment", flush=True)
    rng = np.random.default_rng(99)
    s = rand_stream(rng, 70000, 1, 40, 4)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    assert np.array_equal(gpu_once(torch_cuda, s, 4), want)


def test_accumulate_dump_reset(torch_cuda, oracle_lib):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    rng = np.random.default_rng(5)
    T, F, N = 96, 3, 150
    gulps = [rand_stream(rng, T, F, N, 4) for _ in range(3)]
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T)]) as c:
        # a dump before any data is all zeros
        assert not c.dump()[0].cpu().numpy().any()
        for g in gulps:
            c.correlate([torch.from_numpy(g).cuda()])
        assert c.samples_since_dump() == 3 * T
        # snapshot without reset keeps integrating
        snap = c.dump(reset=False)[0].cpu().numpy()
        acc = np.zeros((F, N * (N + 1) // 2, 2), np.int64)
        for g in gulps:
            oracle_lib.accumulate(acc, g, 4)
        assert np.array_equal(snap, oracle_lib.narrow(acc))
        c.correlate([torch.from_numpy(gulps[0]).cuda()])
        oracle_lib.accumulate(acc, gulps[0], 4)
        host = c.dump(device=False)[0].numpy()
        assert np.array_equal(host, oracle_lib.narrow(acc))
        assert c.samples_since_dump() == 0
        # after the reset the next integration starts from zero
        c.correlate([torch.from_numpy(gulps[1]).cuda()])
        assert np.array_equal(c.dump()[0].cpu().numpy(),
                              oracle_lib.narrow(oracle_lib.correlate(gulps[1], 4)))


def test_repeatable_bits(torch_cuda):
    # integer results do not depend on order: repeated runs give identical bits
    rng = np.random.default_rng(6)
    s = rand_stream(rng, 512, 4, 300, 4)
    a = gpu_once(torch_cuda, s, 4)
    b = gpu_once(torch_cuda, s, 4)
    assert np.array_equal(a, b)


def test_multi_segment_wave_path(torch_cuda, oracle_lib):
    # N a multiple of 16 (wave-persistent kernel), a call of 3 launch segments
    print("case multi-segment wave path", flush=True)
    rng = np.random.default_rng(98)
    s = rand_stream(rng, 70000, 2, 48, 4)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    assert np.array_equal(gpu_once(torch_cuda, s, 4), want)


def test_several_subarrays_one_context(torch_cuda, oracle_lib):
    # subarrays of uneven shape in one context: wave-path ones share one
    # persistent launch, the others take the register-staging kernel
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case several subarrays", flush=True)
    rng = np.random.default_rng(77)
    shapes = [(16, 5, 300, 4), (64, 3, 300, 4), (192, 2, 130, 4), (100, 2, 200, 4), (48, 2, 90, 8)]
    streams = [rand_stream(rng, T, F, N, b) for (N, F, T, b) in shapes]
    subs = [dict(n_inputs=N, n_chans=F, n_time=T, in_bits=b) for (N, F, T, b) in shapes]
    with Correlator(subs) as c:
        dev = [torch.from_numpy(x).cuda() for x in streams]
        c.correlate(dev)
        c.correlate(dev)
        outs = [o.cpu().numpy() for o in c.dump()]
    for (N, F, T, b), x, got in zip(shapes, streams, outs):
        acc = oracle_lib.correlate(x, b)
        want = oracle_lib.narrow(acc * 2)
        assert np.array_equal(got, want), (N, F, T, b)


@pytest.mark.parametrize("code", [-128, 127])
def test_extreme_values_8bit_direct_path(torch_cuda, oracle_lib, code):
    # N a multiple of 8: the 8-bit stream goes through the LDS-copy kernel
    print("case 8-bit extremes N=72 code=%d" % code, flush=True)
    s = np.full((300, 2, 72, 2), code, np.int8)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 8))
    assert np.array_equal(gpu_once(torch_cuda, s, 8), want)


def test_8bit_multi_segment(torch_cuda, oracle_lib):
    # two launch segments of 8-bit input, sums up to the 8-bit dump bound's scale
    print("case 8-bit multi-segment", flush=True)
    rng = np.random.default_rng(97)
    s = rand_stream(rng, 40000, 2, 24, 8)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 8))
    assert np.array_equal(gpu_once(torch_cuda, s, 8), want)

def test_correlate_dump_one_call(torch_cuda, oracle_lib):
    # xeng_correlate_dump: fused into the last launch for the one-wave kernel
    # (the flush adds the accumulator of earlier calls and writes the output),
    # plain correlate + dump for the other kernels; every result exact, the
    # context reset after each call
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case correlate_dump", flush=True)
    rng = np.random.default_rng(41)
    shapes = [(144, 3, 200, 4), (48, 2, 70000, 4), (40, 2, 90, 8), (37, 2, 120, 4)]
    subs = [dict(n_inputs=N, n_chans=F, n_time=T, in_bits=b) for (N, F, T, b) in shapes]
    a = [rand_stream(rng, T, F, N, b) for (N, F, T, b) in shapes]
    b_ = [rand_stream(rng, T, F, N, b) for (N, F, T, b) in shapes]
    with Correlator(subs) as c:
        kinds = [s["kernel"] for s in c.plan()["subarrays"]]
        print("kernels", kinds, flush=True)
        da = [torch.from_numpy(x).cuda() for x in a]
        db = [torch.from_numpy(x).cuda() for x in b_]
        # after an earlier call: sums of both
        c.correlate(da)
        outs = [o.cpu().numpy() for o in c.correlate_dump(db)]
        for (N, F, T, bits), x, y, o in zip(shapes, a, b_, outs):
            want = oracle_lib.narrow(oracle_lib.correlate(x, bits) + oracle_lib.correlate(y, bits))
            assert np.array_equal(o, want), (N, T, bits)
        assert c.samples_since_dump() == 0
        # from a reset context: one call's sums
        outs = [o.cpu().numpy() for o in c.correlate_dump(da)]
        for (N, F, T, bits), x, o in zip(shapes, a, outs):
            assert np.array_equal(o, oracle_lib.narrow(oracle_lib.correlate(x, bits))), (N, T, bits)
        # without reset (not fused): a snapshot, then the integration goes on
        outs = [o.cpu().numpy() for o in c.correlate_dump(db, reset=False)]
        for (N, F, T, bits), y, o in zip(shapes, b_, outs):
            assert np.array_equal(o, oracle_lib.narrow(oracle_lib.correlate(y, bits))), (N, T, bits)
        outs = [o.cpu().numpy() for o in c.correlate_dump(da)]
        for (N, F, T, bits), x, y, o in zip(shapes, a, b_, outs):
            want = oracle_lib.narrow(oracle_lib.correlate(x, bits) + oracle_lib.correlate(y, bits))
            assert np.array_equal(o, want), (N, T, bits)


@pytest.mark.parametrize("kernel", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("N,F,T", [(48, 3, 100), (144, 2, 333), (256, 2, 70000), (512, 1, 257)])
def test_every_kernel_family(torch_cuda, oracle_lib, kernel, N, F, T):
    # each kernel family pinned with xeng_set_kernel: two calls then a dump,
    # then a correlate-and-dump after one call (its flush adds the
    # accumulator's raw sums and writes exact ones), all exact
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case kernel=%d N=%d F=%d T=%d" % (kernel, N, F, T), flush=True)
    rng = np.random.default_rng(kernel * 1000 + N + T)
    a = rand_stream(rng, T, F, N, 4)
    b = rand_stream(rng, T, F, N, 4)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    wa, wb = oracle_lib.correlate(a, 4), oracle_lib.correlate(b, 4)
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T)]) as c:
        c.set_kernel(kernel, tile=64)
        print("plan", c.plan()["subarrays"][0]["kernel"], flush=True)
        c.correlate([da])
        c.correlate([db])
        assert np.array_equal(c.dump()[0].cpu().numpy(), oracle_lib.narrow(wa + wb))
        c.correlate([db])
        got = c.correlate_dump([da])[0].cpu().numpy()
        assert np.array_equal(got, oracle_lib.narrow(wa + wb))
        got = c.correlate_dump([db])[0].cpu().numpy()
        assert np.array_equal(got, oracle_lib.narrow(wb))


@pytest.mark.parametrize("N,F,T", [(384, 300, 200), (256, 600, 64), (128, 1500, 97), (192, 300, 1100)])
def test_diagonal_tiles_many_per_workgroup(torch_cuda, oracle_lib, N, F, T):
    # 4-bit input, persistent kernel: a diagonal tile's blocks are split by K
    # step between waves and the halves meet through LDS at the flush. With
    # many channels every workgroup flushes many diagonal tiles in a row (the
    # hand-over slot and the S_i table are reused); whole and ragged last
    # stages; raw sums (correlate + dump) and exact ones (correlate-and-dump)
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case diagonal K split N=%d F=%d T=%d" % (N, F, T), flush=True)
    rng = np.random.default_rng(N * 7 + F + T)
    s = rand_stream(rng, T, F, N, 4)
    chans = sorted(set([0, 1, F // 2, F - 2, F - 1] + rng.choice(F, 12, replace=False).tolist()))
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4, chans=chans))
    d = torch.from_numpy(s).cuda()
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T)]) as c:
        assert c.plan()["subarrays"][0]["kernel"] == "persistent_workgroup"
        c.correlate([d])
        raw = c.dump()[0][chans].cpu().numpy()
        fused = c.correlate_dump([d])[0][chans].cpu().numpy()
    assert np.array_equal(raw, want)
    assert np.array_equal(fused, want)


@pytest.mark.parametrize("N,F,T", [(64, 5, 100), (64, 1030, 513), (64, 2, 70000), (32, 3, 256),
                                   (16, 7, 1), (48, 4, 1000), (64, 600, 4096)])
def test_small_n_kernel(torch_cuda, oracle_lib, N, F, T):
    # the small-N kernel (one channel per item, the default for 4-bit N <= 64):
    # ragged and whole stages, several channels per workgroup (F above the
    # resident workgroups), several segments, accumulate then correlate-and-dump
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case small_n N=%d F=%d T=%d" % (N, F, T), flush=True)
    rng = np.random.default_rng(7000 + N + F + T)
    a = rand_stream(rng, T, F, N, 4)
    b = rand_stream(rng, T, F, N, 4)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    # full oracle on a channel sample when F is large (first, last, seeded)
    chans = None if F <= 16 else sorted({0, F - 1, *rng.choice(F, 6, replace=False).tolist()})
    wa = oracle_lib.correlate(a, 4, chans=chans)
    wb = oracle_lib.correlate(b, 4, chans=chans)
    pick = (lambda v: v) if chans is None else (lambda v: v[chans])
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T)]) as c:
        assert c.plan()["subarrays"][0]["kernel"] == "small_n"
        c.correlate([da])
        c.correlate([db])
        assert np.array_equal(pick(c.dump()[0].cpu().numpy()), oracle_lib.narrow(wa + wb))
        c.correlate([db])
        got = c.correlate_dump([da])[0].cpu().numpy()
        assert np.array_equal(pick(got), oracle_lib.narrow(wa + wb))
        got = c.correlate_dump([db])[0].cpu().numpy()
        assert np.array_equal(pick(got), oracle_lib.narrow(wb))
        if chans is not None:
            # every channel by the projection check
            wrng = np.random.default_rng(7100 + N + F)
            for f in range(F):
                w = wrng.integers(-4, 5, size=(N, 2)).astype(np.int64)
                assert oracle_lib.projection_check(b, 4, f, got[f], w) == 0, f
