"""Parity at the full sizes of every configuration, in the launch configuration
the benchmark times.

- LEDA gulp (N = 512, 128 channels, 8192 samples, tone in 4 channels): every
  channel against the full oracle.
- Precision variants (N = 512, 256 channels, 16384 samples; FP8 engine on
  4-bit input, int8 engine on 8-bit input): every channel by the projection
  check, sampled channels against the full oracle, and the FP8 engine equal to
  the int8 engine on every word.
- Batch (N = 64 ... 2048, 4096 samples, autotuned, graph replay): every channel
  of every subarray by the projection check, sampled channels in full.
- Stream (N = 512, 2400 channels, 8192-sample gulps through the 4-slot ring,
  one 26-gulp dump): the 4 tone channels and 12 seeded channels against the
  full oracle, 16 more by the projection check, on samples regenerated on the
  host from the same counter-based generator.

The projection check compares V w with sum_t x (x^H w) for a random small-
integer w, exactly in int64: a wrong cell changes V w unless w happens to be
orthogonal to the error. Each test prints how many channels it covered.
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


def run_once(torch, samples, in_bits, engine=0):
    from paper_1411_3751_amd import Correlator
    T, F, N = samples.shape[:3]
    d = torch.from_numpy(samples).cuda()
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits, engine=engine)]) as c:
        c.correlate([d])
        out = c.dump()[0]
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    del d
    return got


def project_all(oracle_lib, samples, in_bits, got, chans, seed):
    """Projection check of every channel in chans; returns the failing ones."""
    N = samples.shape[2]
    rng = np.random.default_rng(seed)
    bad = []
    for f in chans:
        w = rng.integers(-4, 5, size=(N, 2)).astype(np.int64)
        if oracle_lib.projection_check(samples, in_bits, int(f), got[f], w) != 0:
            bad.append(int(f))
    return bad


@pytest.mark.timeout(900)
def test_leda_gulp_every_channel(torch_cuda, oracle_lib):
    print("case leda_gulp N=512 F=128 T=8192, full oracle on all channels", flush=True)
    s, _, _, meta = synth.workload("leda_gulp")
    got = run_once(torch_cuda, s, 4)
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4))
    bad = np.argwhere(got != want)
    print("leda_gulp: %d of %d channels checked in full" % (want.shape[0], meta["n_chans"]), flush=True)
    assert bad.size == 0, "first mismatches %s" % bad[:5].tolist()


@pytest.mark.timeout(900)
def test_fp8_variant_every_channel(torch_cuda, oracle_lib):
    print("case fp8_variant N=512 F=256 T=16384, projection on all channels", flush=True)
    s, _, _, meta = synth.workload("fp8_variant")
    F = meta["n_chans"]
    a = run_once(torch_cuda, s, 4, engine=1)
    b = run_once(torch_cuda, s, 4, engine=0)
    assert np.array_equal(a, b), "FP8 and int8 engines differ"
    rng = np.random.default_rng(3001)
    full = sorted(rng.choice(F, 8, replace=False).tolist())
    want = oracle_lib.narrow(oracle_lib.correlate(s, 4, chans=full))
    assert np.array_equal(a[full], want)
    bad = project_all(oracle_lib, s, 4, a, range(F), 3002)
    print("fp8_variant: %d channels in full, %d of %d by projection" % (len(full), F, F), flush=True)
    assert not bad, "projection fails on channels %s" % bad[:8]


@pytest.mark.timeout(900)
def test_int8_variant_every_channel(torch_cuda, oracle_lib):
    print("case int8_variant N=512 F=256 T=16384 8-bit, projection on all channels", flush=True)
    s, _, _, meta = synth.workload("int8_variant")
    F = meta["n_chans"]
    got = run_once(torch_cuda, s, 8)
    rng = np.random.default_rng(3003)
    full = sorted(rng.choice(F, 8, replace=False).tolist())
    want = oracle_lib.narrow(oracle_lib.correlate(s, 8, chans=full))
    assert np.array_equal(got[full], want)
    bad = project_all(oracle_lib, s, 8, got, range(F), 3004)
    print("int8_variant: %d channels in full, %d of %d by projection" % (len(full), F, F), flush=True)
    assert not bad, "projection fails on channels %s" % bad[:8]


@pytest.mark.timeout(900)
def test_batch_every_channel(torch_cuda, oracle_lib):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case batch N=64..2048 T=4096, autotuned graph replay, projection on all channels",
          flush=True)
    streams, subs = [], []
    for k in range(len(synth.BATCH_SHAPES)):
        x, _, _, meta = synth.workload("batch", subarray=k)
        streams.append(x)
        subs.append(dict(n_inputs=meta["n_inputs"], n_chans=meta["n_chans"], n_time=meta["n_time"]))
    dev = [torch.from_numpy(x).cuda() for x in streams]
    out = [torch.empty((d["n_chans"], d["n_inputs"] * (d["n_inputs"] + 1) // 2, 2),
                       dtype=torch.int32, device="cuda") for d in subs]
    with Correlator(subs) as c:
        c.autotune(dev, reps=2)
        print("plan", c.plan(), flush=True)
        with c.capture(dev, out) as g:
            for _ in range(2):
                g.launch()
            torch.cuda.synchronize()
    rng = np.random.default_rng(3005)
    for k, (x, d, o) in enumerate(zip(streams, subs, out)):
        N, F = d["n_inputs"], d["n_chans"]
        got = o.cpu().numpy()
        full = sorted(rng.choice(F, min(F, 4), replace=False).tolist())
        want = oracle_lib.narrow(oracle_lib.correlate(x, 4, chans=full))
        assert np.array_equal(got[full], want), N
        bad = project_all(oracle_lib, x, 4, got, range(F), 3006 + k)
        print("batch N=%d: %d channels in full, %d of %d by projection" % (N, len(full), F, F),
              flush=True)
        assert not bad, "N=%d: projection fails on channels %s" % (N, bad[:8])


@pytest.mark.timeout(900)
def test_stream_configuration_one_dump(torch_cuda, oracle_lib):
    # N = 512, 2400 channels, 8192-sample gulps of the drifting-tone stream
    # into a 4-slot ring, dump after 26 gulps to pinned host memory
    import synth.gpu
    from paper_1411_3751_amd import Stream
    torch = torch_cuda
    synth.gpu.build()
    N, F, T, every, slots = 512, 2400, 8192, 26, 4
    print("case stream N=%d F=%d T=%d, %d-gulp dump through a %d-slot ring" % (N, F, T, every, slots),
          flush=True)
    seed = synth.SEED_BASE + 4
    tone = (synth.TONE_AMP, lambda t: synth.drift_phase(t, T), synth.tone_channels(F))
    gen = synth.gpu.DeviceStream(seed, F, N, 4, 2.5, tone=tone, t_total=every * T)
    tri = N * (N + 1) // 2
    hd = [torch.empty((F, tri, 2), dtype=torch.int32, pin_memory=True)]
    with Stream(dict(n_inputs=N, n_chans=F, n_time=T), n_slots=slots, dump_every=every,
                host_dumps=hd) as st:
        for g in range(every):
            ptr, ist = st.next_slot()
            gen.fill(ptr, g * T, T, ist)
            st.push()
        st.dump_wait(0)
        got = hd[0].numpy()
    rng = np.random.default_rng(3011)
    tch = synth.tone_channels(F)
    rest = [f for f in range(F) if f not in tch]
    picks = rng.choice(rest, 28, replace=False).tolist()
    full = tch + sorted(picks[:12])
    proj = sorted(picks[12:])
    x, _, _ = synth.stream(seed, every * T, F, N, 4, 2.5, chans=full + proj, tone=tone)
    xf = np.ascontiguousarray(x[:, :len(full)])
    want = oracle_lib.narrow(oracle_lib.correlate(xf, 4))
    del xf
    bad = np.argwhere(got[full] != want)
    assert bad.size == 0, "first mismatches (channel index in %s) %s" % (full, bad[:5].tolist())
    xp = np.ascontiguousarray(x[:, len(full):])
    del x
    wrng = np.random.default_rng(3012)
    for k, f in enumerate(proj):
        w = wrng.integers(-4, 5, size=(N, 2)).astype(np.int64)
        assert oracle_lib.projection_check(xp, 4, k, got[f], w) == 0, f
    # the tone channels carry the common tone: Re V_ij / T near |A|^2 off the
    # diagonal (a sanity check of the channel order, not parity)
    v = got[tch[0], :, 0].astype(np.float64) / (every * T)
    ii, jj = np.tril_indices(N, -1)
    assert abs(np.mean(v[ii * (ii + 1) // 2 + jj]) - synth.TONE_AMP ** 2) < 0.3
    print("stream: %d channels in full, %d by projection, of %d" % (len(full), len(proj), F),
          flush=True)
