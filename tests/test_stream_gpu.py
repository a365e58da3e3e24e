"""Streaming integration through the device gulp ring (xeng_stream_*), and the
GPU side of the input generator.

Gulps are produced on the device by the counter-based generator (a drifting
common tone, phase-continuous across gulps), pushed through a 4-slot ring and
dumped every few gulps; each dump must equal the oracle's sums over exactly
the gulps of its period, regenerated on the host.
"""
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
    import synth.gpu
    synth.gpu.build()
    return torch


def drift_tone(F, gulp):
    return (synth.TONE_AMP, lambda t: synth.drift_phase(t, gulp), synth.tone_channels(F))


@pytest.mark.parametrize("in_bits,N", [(4, 48), (8, 40), (4, 37)])
def test_gpu_generator_matches_host(torch_cuda, in_bits, N):
    import synth.gpu
    torch = torch_cuda
    print("case generator in_bits=%d N=%d" % (in_bits, N), flush=True)
    T, F, t0, seed = 300, 16, 5000, 4242
    sigma = 2.5 if in_bits == 4 else 20.0
    tone = drift_tone(F, 128)
    gen = synth.gpu.DeviceStream(seed, F, N, in_bits, sigma, tone=tone, t_total=t0 + T)
    shape = (T, F, N) if in_bits == 4 else (T, F, N, 2)
    buf = torch.empty(shape, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    gen.fill(buf.data_ptr(), t0, T, s.cuda_stream)
    torch.cuda.synchronize()
    want, _, _ = synth.stream(seed, T, F, N, in_bits, sigma, t0=t0, tone=tone)
    got = buf.cpu().numpy()
    if in_bits == 8:
        got = got.view(np.int8)
    assert np.array_equal(got, want)


def run_stream(torch, N, F, T, n_gulps, dump_every, in_bits=4, host=True):
    import synth.gpu
    from paper_1411_3751_amd import Stream
    seed = 99
    sigma = 2.5 if in_bits == 4 else 20.0
    tone = drift_tone(F, T)
    gen = synth.gpu.DeviceStream(seed, F, N, in_bits, sigma, tone=tone, t_total=n_gulps * T)
    shape = (F, N * (N + 1) // 2, 2)
    hd = [torch.empty(shape, dtype=torch.int32, pin_memory=True) for _ in range(2)] if host else None
    sub = dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits)
    dumps, times = [], []
    with Stream(sub, n_slots=4, dump_every=dump_every, host_dumps=hd) as st:
        for g in range(n_gulps):
            ptr, ist = st.next_slot()
            gen.fill(ptr, g * T, T, ist)
            st.push()
            if (g + 1) % dump_every == 0:
                d = (g + 1) // dump_every - 1
                dp = st.dump_wait(d)
                if host:
                    dumps.append(hd[d % 2].numpy().copy())
                else:
                    h = np.empty(shape, np.int32)
                    hip = ctypes.CDLL("libamdhip64.so")
                    assert hip.hipMemcpy(ctypes.c_void_p(h.ctypes.data), ctypes.c_void_p(dp),
                                         ctypes.c_size_t(h.nbytes), 2) == 0
                    dumps.append(h)
        for g in range(n_gulps):
            times.append(st.gulp_times(g))
        assert st.gulps() == n_gulps
    return dumps, times, seed, sigma, tone


@pytest.mark.parametrize("host", [True, False])
def test_stream_dumps_match_oracle(torch_cuda, oracle_lib, host):
    print("case stream host=%s" % host, flush=True)
    N, F, T, dump_every, n_gulps = 128, 16, 2048, 3, 7
    dumps, times, seed, sigma, tone = run_stream(torch_cuda, N, F, T, n_gulps, dump_every,
                                                 host=host)
    assert len(dumps) == 2
    for d, got in enumerate(dumps):
        x, _, _ = synth.stream(seed, dump_every * T, F, N, 4, sigma, t0=d * dump_every * T,
                               tone=tone)
        want = oracle_lib.narrow(oracle_lib.correlate(x, 4))
        bad = np.argwhere(got != want)
        assert bad.size == 0, "dump %d first mismatches %s" % (d, bad[:5].tolist())
    for a, r in times:
        assert a >= r > 0


def test_stream_8bit_and_odd_n(torch_cuda, oracle_lib):
    # 8-bit gulps with N not a multiple of 8 take the register-staging kernel
    print("case stream 8-bit N=30", flush=True)
    N, F, T, dump_every, n_gulps = 30, 8, 1000, 2, 4
    dumps, _, seed, sigma, tone = run_stream(torch_cuda, N, F, T, n_gulps, dump_every, in_bits=8)
    for d, got in enumerate(dumps):
        x, _, _ = synth.stream(seed, dump_every * T, F, N, 8, sigma, t0=d * dump_every * T,
                               tone=tone)
        assert np.array_equal(got, oracle_lib.narrow(oracle_lib.correlate(x, 8)))


def test_stream_errors(torch_cuda):
    from paper_1411_3751_amd import Stream, XengError
    from paper_1411_3751_amd.xeng import XENG_EINVAL, XENG_ERANGE
    sub = dict(n_inputs=16, n_chans=2, n_time=64)
    with pytest.raises(XengError) as ei:
        Stream(sub, n_slots=1)
    assert ei.value.code == XENG_EINVAL
    with pytest.raises(XengError) as ei:
        Stream(dict(n_inputs=16, n_chans=2, n_time=40000, in_bits=8), n_slots=2, dump_every=2)
    assert ei.value.code == XENG_ERANGE
    with Stream(sub, n_slots=2, dump_every=2) as st:
        with pytest.raises(XengError) as ei:
            st.push()
        assert ei.value.code == XENG_EINVAL
        with pytest.raises(XengError) as ei:
            st.dump_wait(0)
        assert ei.value.code == XENG_EINVAL


def test_stream_drops_and_fast_autos(torch_cuda, oracle_lib):
    # gulps 5 and 7 are dropped (7 ends dump 1): every dump covers the same
    # span of gulps and sums only the pushed ones; the autocorrelations of 4
    # selected inputs are dumped and cleared every 2 gulps inside the stream
    import synth.gpu
    from paper_1411_3751_amd import Stream
    torch = torch_cuda
    print("case stream drops + fast autos", flush=True)
    N, F, T, every, fast_every, n_gulps = 64, 8, 512, 4, 2, 10
    sel = [0, 3, 17, 63]
    drops = {5, 7}
    seed, sigma = 77, 2.5
    tone = drift_tone(F, T)
    gen = synth.gpu.DeviceStream(seed, F, N, 4, sigma, tone=tone, t_total=n_gulps * T)
    shape = (F, N * (N + 1) // 2, 2)
    hd = [torch.empty(shape, dtype=torch.int32, pin_memory=True) for _ in range(3)]
    fh = [torch.empty((F, len(sel)), dtype=torch.int32, pin_memory=True) for _ in range(6)]
    with Stream(dict(n_inputs=N, n_chans=F, n_time=T), n_slots=3, dump_every=every,
                host_dumps=hd) as st:
        st.set_fast_autos(sel, fast_every, host_out=fh)
        for g in range(n_gulps):
            if g in drops:
                assert st.drop() == g
                continue
            ptr, ist = st.next_slot()
            gen.fill(ptr, g * T, T, ist)
            st.push()
        st.dump_wait(1)
        st.fast_wait(4)
        stats = st.stats()
        dumps = [hd[d].numpy().copy() for d in range(2)]
        fasts = [fh[k].numpy().copy() for k in range(5)]
    assert stats["gulps"] == n_gulps and stats["dropped"] == 2 and stats["correlated"] == 8
    assert stats["dumps"] == 2 and stats["fast_dumps"] == 5
    per_gulp = []
    for g in range(n_gulps):
        x, _, _ = synth.stream(seed, T, F, N, 4, sigma, t0=g * T, tone=tone)
        per_gulp.append(oracle_lib.correlate(x, 4) if g not in drops else None)
    diag = [i * (i + 1) // 2 + i for i in sel]
    for d in range(2):
        acc = sum(per_gulp[g] for g in range(d * every, (d + 1) * every) if g not in drops)
        want = oracle_lib.narrow(acc)
        # every main dump here falls on a fast dump, which cleared the selected autos
        want[:, diag, 0] = 0
        assert np.array_equal(dumps[d], want), d
    for k in range(5):
        acc = sum(per_gulp[g] for g in range(k * fast_every, (k + 1) * fast_every) if g not in drops)
        assert np.array_equal(fasts[k], acc[:, diag, 0].astype(np.int32)), k


def test_stream_nonblocking_drops_are_counted_and_exact(torch_cuda, oracle_lib):
    # a slow producer on the ingest stream keeps the two slots busy: in
    # non-blocking mode next_slot drops gulps instead of waiting; whichever
    # gulps were dropped, each dump equals the oracle over the pushed ones
    import synth.gpu
    from paper_1411_3751_amd import Stream
    torch = torch_cuda
    print("case stream non-blocking overload", flush=True)
    N, F, T, every, n_gulps = 128, 16, 4096, 6, 24
    seed, sigma = 78, 2.5
    tone = drift_tone(F, T)
    gen = synth.gpu.DeviceStream(seed, F, N, 4, sigma, tone=tone, t_total=n_gulps * T)
    slow = synth.gpu.DeviceStream(seed + 1, 512, 4096, 4, sigma, tone=None, t_total=256)
    ballast = torch.empty((256, 512, 4096), dtype=torch.uint8, device="cuda")
    shape = (F, N * (N + 1) // 2, 2)
    hd = [torch.empty(shape, dtype=torch.int32, pin_memory=True) for _ in range(4)]
    pushed = []
    with Stream(dict(n_inputs=N, n_chans=F, n_time=T), n_slots=2, dump_every=every,
                host_dumps=hd) as st:
        st.set_nonblocking(True)
        for g in range(n_gulps):
            ptr, ist = st.next_slot()
            if ptr is None:
                continue
            slow.fill(ballast.data_ptr(), 0, 256, ist)  # a producer that takes a while
            gen.fill(ptr, g * T, T, ist)
            st.push()
            pushed.append(g)
        st.dump_wait(n_gulps // every - 1)
        stats = st.stats()
        got = [hd[d].numpy().copy() for d in range(n_gulps // every)]
    print("pushed", pushed, "stats", stats, flush=True)
    assert stats["gulps"] == n_gulps
    assert stats["correlated"] == len(pushed) and stats["dropped"] == n_gulps - len(pushed)
    assert stats["dropped"] > 0, "the slow producer should have made some gulps late"
    for d in range(n_gulps // every):
        gs = [g for g in pushed if d * every <= g < (d + 1) * every]
        acc = np.zeros((F, N * (N + 1) // 2, 2), np.int64)
        for g in gs:
            x, _, _ = synth.stream(seed, T, F, N, 4, sigma, t0=g * T, tone=tone)
            oracle_lib.accumulate(acc, x, 4)
        assert np.array_equal(got[d], oracle_lib.narrow(acc)), d
