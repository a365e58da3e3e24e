"""Pins of the reference packet corner turn (CPU): it must invert the
packetizer exactly, and drop, duplicate and reject packets as stated."""
import numpy as np

import synth
from oracle.ingest import depacketize


def setup(in_bits=4, T=8, F=6, N=12, pt=2, pc=3, pi=4, seed=1):
    rng = np.random.default_rng(seed)
    if in_bits == 4:
        s = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
    else:
        s = rng.integers(-128, 128, size=(T, F, N, 2)).astype(np.int8)
    t0 = 4096
    pk = synth.packetize(s, t0, pt, pc, pi, in_bits)
    return s, t0, pk, rng


def flat(s):
    return np.ascontiguousarray(s).view(np.uint8).reshape(s.shape[0], s.shape[1], -1)


def test_round_trip_any_order():
    for in_bits in (4, 8):
        s, t0, pk, rng = setup(in_bits)
        perm = rng.permutation(len(pk))
        g, st = depacketize(pk[perm], 8, 6, 12, in_bits, t0, 2, 3, 4)
        assert np.array_equal(g, flat(s))
        assert st == dict(received=len(pk), missing=0, duplicate=0, rejected=0)


def test_header_fields():
    s, t0, pk, _ = setup()
    # packet (time block 1, channel block 1, input block 2)
    k = (1 * 2 + 1) * 3 + 2
    h = pk[k, :16]
    assert int.from_bytes(bytes(h[0:8]), "little") == t0 + 2
    assert int.from_bytes(bytes(h[8:10]), "little") == 3
    assert int.from_bytes(bytes(h[10:12]), "little") == 8
    assert int.from_bytes(bytes(h[12:16]), "little") == synth.PACKET_MAGIC
    assert np.array_equal(pk[k, 16:16 + 24].reshape(2, 3, 4), s[2:4, 3:6, 8:12])


def test_missing_blocks_are_zero():
    s, t0, pk, rng = setup()
    keep = np.ones(len(pk), bool)
    keep[[0, 5, 17]] = False
    g, st = depacketize(pk[keep], 8, 6, 12, 4, t0, 2, 3, 4)
    want = s.copy()
    for k in (0, 5, 17):
        tb, fb, ib = k // 6, (k // 3) % 2, k % 3
        want[2 * tb:2 * tb + 2, 3 * fb:3 * fb + 3, 4 * ib:4 * ib + 4] = 0
    assert np.array_equal(g, want)
    assert st["missing"] == 3 and st["received"] == len(pk) - 3


def test_duplicates_and_rejects():
    s, t0, pk, rng = setup()
    bad = pk[:4].copy()
    bad[0, 12] ^= 1                                       # magic
    bad[1, 0:8] = np.frombuffer(np.uint64(t0 + 1).tobytes(), np.uint8)   # misaligned time
    bad[2, 0:8] = np.frombuffer(np.uint64(t0 + 8).tobytes(), np.uint8)   # outside the gulp
    bad[3, 8:10] = np.frombuffer(np.uint16(1).tobytes(), np.uint8)       # misaligned channel
    dup = pk[[3, 3, 7]]
    g, st = depacketize(np.concatenate([pk, bad, dup]), 8, 6, 12, 4, t0, 2, 3, 4)
    assert np.array_equal(g, s)
    assert st == dict(received=len(pk), missing=0, duplicate=3, rejected=4)
