"""C-ABI argument checks that run before any HIP call, so they hold on a host
without a GPU: every create call refuses bad shapes, sizes past the 32-bit
offset and exactness limits, and bad F-engine, stream and ingest settings
with XENG_EINVAL or XENG_ERANGE and a message, and allocates nothing."""
import ctypes
import math
import os

import pytest

from paper_1411_3751_amd import xeng

pytestmark = pytest.mark.skipif(not os.path.exists(xeng.LIB_PATH), reason="libxeng.so not built")


def sub(n_inputs, n_chans, n_time, in_bits=4, engine=0):
    return xeng.Subarray(n_inputs, n_chans, n_time, in_bits, engine)


def create(*subs, n=None):
    lib = xeng.load()
    arr = (xeng.Subarray * max(len(subs), 1))(*subs)
    ctx = ctypes.c_void_p(12345)
    rc = lib.xeng_create(arr, len(subs) if n is None else n, None, ctypes.byref(ctx))
    return rc, ctx.value, lib.xeng_last_error().decode()


@pytest.mark.parametrize("bad, words", [
    (sub(0, 1, 1), "n_inputs"),
    (sub(65536, 1, 1), "n_inputs"),
    (sub(4, 0, 1), "n_chans"),
    (sub(4, 1 << 24, 1), "n_chans"),
    (sub(4, 1, 0), "n_time"),
    (sub(4, 1, 8, in_bits=6), "in_bits"),
    (sub(4, 1, 8, engine=7), "engine"),
    (sub(16, 1, 8, in_bits=8, engine=1), "4-bit"),
    (sub(40, 1, 8, in_bits=4, engine=1), "multiple of 16"),
])
def test_create_rejects_bad_subarrays(bad, words):
    rc, ctx, msg = create(bad)
    assert rc == xeng.XENG_EINVAL
    assert ctx is None  # *out cleared, nothing allocated
    assert words in msg


def test_create_rejects_subarray_counts():
    assert create(sub(4, 1, 8), n=0)[0] == xeng.XENG_EINVAL
    many = [sub(4, 1, 8)] * 17
    rc, _, msg = create(*many)
    assert rc == xeng.XENG_EINVAL and "n_subs" in msg


def test_create_rejects_null_arguments():
    lib = xeng.load()
    ctx = ctypes.c_void_p()
    assert lib.xeng_create(None, 1, None, ctypes.byref(ctx)) == xeng.XENG_EINVAL
    arr = (xeng.Subarray * 1)(sub(4, 1, 8))
    assert lib.xeng_create(arr, 1, None, None) == xeng.XENG_EINVAL


def test_bad_subarray_later_in_the_list_is_named():
    rc, _, msg = create(sub(16, 2, 8), sub(16, 2, 8), sub(0, 2, 8))
    assert rc == xeng.XENG_EINVAL
    assert "subarray 2" in msg


def test_32_bit_stage_offsets_are_guarded():
    # one stage spans 64 time rows of the [F][N] plane; its byte offsets must
    # stay below 2^31: F N 64 = 2^31 is refused (one channel less would pass
    # this check; it is not created here, its accumulator is 550 GB)
    assert 8192 * 4096 * 64 == 2 ** 31 and 8191 * 4096 * 64 < 2 ** 31
    rc, _, msg = create(sub(4096, 8192, 8))
    assert rc == xeng.XENG_EINVAL and "too large" in msg
    rc, _, msg = create(sub(2048, 8192, 8, in_bits=8))
    assert rc == xeng.XENG_EINVAL and "too large" in msg


def test_exactness_limit_on_samples_per_call():
    # 4-bit: 128 T < 2^31 ; 8-bit: 32768 T < 2^31
    assert xeng.XENG_ERANGE != xeng.XENG_EINVAL
    rc, _, msg = create(sub(4, 1, 16777216))
    assert rc == xeng.XENG_EINVAL and "dump limit" in msg
    rc, _, msg = create(sub(4, 1, 65536, in_bits=8))
    assert rc == xeng.XENG_EINVAL and "dump limit" in msg
    assert 128 * 16777215 < 2 ** 31 <= 128 * 16777216
    assert 32768 * 65535 < 2 ** 31 <= 32768 * 65536


@pytest.mark.parametrize("cfg, words", [
    ((0, 0, 16, 1.0), "n_inputs"),
    ((65536, 0, 16, 1.0), "n_inputs"),
    ((4, -1, 16, 1.0), "channels"),
    ((4, 4090, 7, 1.0), "channels"),
    ((4, 0, 0, 1.0), "channels"),
    ((4, 0, 16, 0.0), "gain"),
    ((4, 0, 16, -2.0), "gain"),
    ((4, 0, 16, math.inf), "gain"),
    ((4, 0, 16, math.nan), "gain"),
])
def test_fengine_create_rejects_bad_configs(cfg, words):
    lib = xeng.load()
    c = xeng.FEngineConfig(*cfg)
    fe = ctypes.c_void_p(777)
    rc = lib.xeng_fengine_create(ctypes.byref(c), ctypes.byref(fe))
    assert rc == xeng.XENG_EINVAL
    assert fe.value is None
    assert words in lib.xeng_last_error().decode()


def stream_create(s, n_slots=4, dump_every=26, host=None, n_host=0):
    lib = xeng.load()
    out = ctypes.c_void_p(99)
    rc = lib.xeng_stream_create(ctypes.byref(s), n_slots, dump_every, host, n_host, ctypes.byref(out))
    return rc, out.value, lib.xeng_last_error().decode()


def test_stream_create_rejects_bad_settings():
    s = sub(16, 4, 8192)
    assert stream_create(s, n_slots=1)[0] == xeng.XENG_EINVAL
    assert stream_create(s, dump_every=0)[0] == xeng.XENG_EINVAL
    assert stream_create(sub(0, 4, 8192))[0] == xeng.XENG_EINVAL
    # host buffers announced but none given, and a NULL entry among them
    bufs = (ctypes.c_void_p * 2)(None, None)
    assert stream_create(s, host=bufs, n_host=0)[0] == xeng.XENG_EINVAL
    rc, out, msg = stream_create(s, host=bufs, n_host=2)
    assert rc == xeng.XENG_EINVAL and "NULL" in msg and out is None


def test_stream_dump_period_beyond_the_exactness_limit():
    # 4-bit: 2048 gulps of 8192 samples = 16,777,216 > 16,777,215
    rc, out, msg = stream_create(sub(16, 4, 8192), dump_every=2048)
    assert rc == xeng.XENG_ERANGE and out is None and "dump limit" in msg
    # 8-bit: 8 gulps of 8192 = 65,536 > 65,535
    rc, _, _ = stream_create(sub(16, 4, 8192, in_bits=8), dump_every=8)
    assert rc == xeng.XENG_ERANGE


def ingest_create(s, pt, pc, pi):
    lib = xeng.load()
    fmt = xeng.PacketFormat(pt, pc, pi)
    out = ctypes.c_void_p(5)
    rc = lib.xeng_ingest_create(ctypes.byref(s), ctypes.byref(fmt), ctypes.byref(out))
    return rc, out.value, lib.xeng_last_error().decode()


@pytest.mark.parametrize("blocks, words", [
    ((0, 4, 16), ">= 1"),
    ((8, 0, 16), ">= 1"),
    ((7, 4, 16), "divide"),
    ((8, 3, 16), "divide"),
    ((8, 4, 5), "divide"),
])
def test_ingest_create_rejects_bad_packet_blocks(blocks, words):
    rc, out, msg = ingest_create(sub(16, 4, 64), *blocks)
    assert rc == xeng.XENG_EINVAL and out is None
    assert words in msg


def test_ingest_create_rejects_bad_subarray():
    rc, _, msg = ingest_create(sub(16, 0, 64), 8, 1, 16)
    assert rc == xeng.XENG_EINVAL and "n_chans" in msg


def test_error_strings():
    lib = xeng.load()
    for code in (xeng.XENG_OK, xeng.XENG_EINVAL, xeng.XENG_ERANGE):
        s = lib.xeng_strerror(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.xeng_strerror(xeng.XENG_EINVAL) != lib.xeng_strerror(xeng.XENG_ERANGE)
