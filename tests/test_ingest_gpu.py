"""GPU packet ingest (corner turn + drop accounting) against the reference
depacketizer, byte for byte, and feeding the correlator."""
import numpy as np
import pytest

import synth
from oracle.ingest import depacketize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_packets(rng, s, t0, fmt, in_bits, drop=0.1, dup=0.05, bad=6):
    pk = synth.packetize(s, t0, *fmt, in_bits)
    keep = rng.random(len(pk)) >= drop
    parts = [pk[keep], pk[rng.choice(len(pk), int(dup * len(pk)), replace=False)]]
    if bad:
        b = pk[rng.choice(len(pk), bad, replace=False)].copy()
        b[0::3, 12] ^= 0x5A                                                   # magic
        b[1::3, 0:8] = np.frombuffer(np.uint64(t0 + s.shape[0]).tobytes(), np.uint8)  # past the gulp
        b[2::3, 10:12] = np.frombuffer(np.uint16(1).tobytes(), np.uint8)      # misaligned input
        parts.append(b)
    allp = np.concatenate(parts)
    return np.ascontiguousarray(allp[rng.permutation(len(allp))])


CASES = [
    # (in_bits, T, F, N, (pkt_time, pkt_chans, pkt_inputs))  copy unit 16 / 4 / 1 / 16
    (4, 64, 8, 64, (4, 2, 32)),
    (4, 32, 6, 48, (2, 3, 4)),
    (4, 30, 4, 30, (3, 2, 3)),
    (8, 32, 4, 40, (4, 2, 8)),
]


@pytest.mark.parametrize("in_bits,T,F,N,fmt", CASES)
def test_ingest_matches_reference(torch_cuda, in_bits, T, F, N, fmt):
    from paper_1411_3751_amd import Ingest
    torch = torch_cuda
    print("case ingest in_bits=%d T=%d F=%d N=%d fmt=%s" % (in_bits, T, F, N, fmt), flush=True)
    rng = np.random.default_rng(T + F + N + in_bits)
    sub = dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits)
    shape = (T, F, N) if in_bits == 4 else (T, F, N, 2)
    with Ingest(sub, *fmt) as ig:
        assert ig.stride == synth.packet_stride(*fmt, in_bits)
        for g in range(2):                       # two gulps: state is cleared per gulp
            t0 = 1000 * T + g * T
            if in_bits == 4:
                s = rng.integers(0, 256, size=shape, dtype=np.uint8)
            else:
                s = rng.integers(-128, 128, size=shape).astype(np.int8)
            pk = make_packets(rng, s, t0, fmt, in_bits)
            want, wst = depacketize(pk, T, F, N, in_bits, t0, *fmt)
            d_pk = torch.from_numpy(pk.reshape(-1)).cuda()
            out = torch.full(shape, 0x77, dtype=torch.uint8, device="cuda")
            ig.gulp(d_pk, len(pk), t0, out)
            got = out.cpu().numpy().reshape(T, F, -1)
            assert np.array_equal(got, want)
            assert ig.stats() == wst


def test_ingest_then_correlate(torch_cuda, oracle_lib):
    # packets of a quantised-Gaussian gulp, 10 % lost: the correlation of the
    # ingested gulp equals the oracle's correlation of the reference gulp
    from paper_1411_3751_amd import Correlator, Ingest
    torch = torch_cuda
    print("case ingest + correlate", flush=True)
    T, F, N, fmt = 256, 8, 128, (8, 4, 32)
    s, _, _, _ = synth.workload("leda_gulp", n_time=T, n_chans=F, n_inputs=N)
    rng = np.random.default_rng(9)
    t0 = 77 * T
    pk = make_packets(rng, s, t0, fmt, 4)
    ref, st = depacketize(pk, T, F, N, 4, t0, *fmt)
    assert st["missing"] > 0
    sub = dict(n_inputs=N, n_chans=F, n_time=T)
    gulp = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
    with Ingest(sub, *fmt) as ig, Correlator([sub]) as c:
        ig.gulp(torch.from_numpy(pk.reshape(-1)).cuda(), len(pk), t0, gulp)
        c.correlate([gulp])
        got = c.dump()[0].cpu().numpy()
    assert np.array_equal(got, oracle_lib.narrow(oracle_lib.correlate(ref.reshape(T, F, N), 4)))


def test_ingest_errors(torch_cuda):
    from paper_1411_3751_amd import Ingest, XengError
    from paper_1411_3751_amd.xeng import XENG_EINVAL
    with pytest.raises(XengError) as ei:
        Ingest(dict(n_inputs=48, n_chans=6, n_time=32), 3, 3, 4)   # 3 does not divide 32
    assert ei.value.code == XENG_EINVAL


def test_ingest_duplicates_with_different_payloads(torch_cuda):
    # retransmitted blocks whose payloads differ: the first copy in buffer
    # order fills the block (as the reference does), run after run
    from paper_1411_3751_amd import Ingest
    torch = torch_cuda
    print("case ingest differing duplicates", flush=True)
    T, F, N, fmt = 64, 8, 64, (4, 2, 32)
    rng = np.random.default_rng(12)
    s = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
    t0 = 5000
    pk = synth.packetize(s, t0, *fmt, 4)
    # three more copies of 40 blocks, each with its own random payload
    extra = []
    for _ in range(3):
        e = pk[rng.choice(len(pk), 40, replace=False)].copy()
        e[:, 16:] = rng.integers(0, 256, size=e[:, 16:].shape, dtype=np.uint8)
        extra.append(e)
    allp = np.concatenate([pk] + extra)
    allp = np.ascontiguousarray(allp[rng.permutation(len(allp))])
    want, wst = depacketize(allp, T, F, N, 4, t0, *fmt)
    assert wst["duplicate"] == 120
    sub = dict(n_inputs=N, n_chans=F, n_time=T)
    d_pk = torch.from_numpy(allp.reshape(-1)).cuda()
    with Ingest(sub, *fmt) as ig:
        for rep in range(3):
            out = torch.full((T, F, N), 0x55, dtype=torch.uint8, device="cuda")
            ig.gulp(d_pk, len(allp), t0, out)
            assert np.array_equal(out.cpu().numpy(), want), rep
            assert ig.stats() == wst


def test_ingest_gulps_on_two_streams(torch_cuda):
    # successive gulps of one engine on different streams are ordered: each
    # gulp's counters and bytes are its own
    from paper_1411_3751_amd import Ingest
    torch = torch_cuda
    print("case ingest two streams", flush=True)
    T, F, N, fmt = 64, 8, 64, (4, 2, 32)
    rng = np.random.default_rng(13)
    sub = dict(n_inputs=N, n_chans=F, n_time=T)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    with Ingest(sub, *fmt) as ig:
        for g in range(4):
            s = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
            t0 = g * T
            pk = make_packets(rng, s, t0, fmt, 4)
            want, wst = depacketize(pk, T, F, N, 4, t0, *fmt)
            st = streams[g % 2]
            with torch.cuda.stream(st):
                d_pk = torch.from_numpy(pk.reshape(-1)).to("cuda", non_blocking=False)
                out = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
            st.synchronize()
            ig.gulp(d_pk, len(pk), t0, out, stream=st)
            assert ig.stats() == wst
            st.synchronize()
            assert np.array_equal(out.cpu().numpy(), want)
