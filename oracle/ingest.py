"""Reference corner turn of F-engine packets into a gulp (test infrastructure only).

Nothing in the product path may import this module. It states, one packet at
a time, what the library's packet ingest must produce: Section 2.3 (the
F-engine boards send packets of a header and channelised samples), Section
2.4 (the CPU layer captures them and completes the corner turn into
[time][channel][input] order; lost packets are counted and not corrected).
The header layout is the library's own (include/xeng.h): little-endian
uint64 first time sample, uint16 first channel, uint16 first input, uint32
magic; the payload is [pkt_time][pkt_chans][pkt_inputs] samples.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x4C454441


def depacketize(packets: np.ndarray, n_time: int, n_chans: int, n_inputs: int, in_bits: int,
                gulp_t0: int, pkt_time: int, pkt_chans: int, pkt_inputs: int):
    """Returns (gulp bytes [T][F][N*bps], stats dict). Packets are processed in
    the given order; the first copy of a block wins."""
    bps = in_bits // 4
    gulp = np.zeros((n_time, n_chans, n_inputs * bps), np.uint8)
    seen = set()
    st = dict(received=0, missing=0, duplicate=0, rejected=0)
    payload = pkt_time * pkt_chans * pkt_inputs * bps
    for pk in packets:
        t0 = int.from_bytes(bytes(pk[0:8]), "little")
        chan0 = int.from_bytes(bytes(pk[8:10]), "little")
        input0 = int.from_bytes(bytes(pk[10:12]), "little")
        magic = int.from_bytes(bytes(pk[12:16]), "little")
        dt = t0 - gulp_t0
        if (magic != MAGIC or not (0 <= dt < n_time) or dt % pkt_time
                or chan0 >= n_chans or chan0 % pkt_chans or input0 >= n_inputs or input0 % pkt_inputs):
            st["rejected"] += 1
            continue
        key = (dt, chan0, input0)
        if key in seen:
            st["duplicate"] += 1
            continue
        seen.add(key)
        st["received"] += 1
        block = np.asarray(pk[16:16 + payload]).reshape(pkt_time, pkt_chans, pkt_inputs * bps)
        for a in range(pkt_time):
            for c in range(pkt_chans):
                gulp[dt + a, chan0 + c, input0 * bps:(input0 + pkt_inputs) * bps] = block[a, c]
    expected = (n_time // pkt_time) * (n_chans // pkt_chans) * (n_inputs // pkt_inputs)
    st["missing"] = expected - st["received"]
    return gulp, st
