"""X-engine benchmark: one JSON line on stdout.

A step is one pass of the whole hot path over one gulp already resident in
HBM: xeng_correlate (unpack, triangle schedule, int8-MFMA cross-multiply,
integration into the int32 accumulator) followed by xeng_dump (device copy of
the packed lower triangle and reset). The workload is the LEDA-shaped gulp:
N = 512 inputs, 128 channels, 8192 samples of 4+4-bit quantised Gaussian
voltages (sigma 2.5) with a common tone in 4 channels.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("complex MACs/s (Tops/s) at N=512, % int8 MFMA peak; real-time factor; "
          "p99 gulp ms")
OPS_PER_CMAC = 8                 # 4 real multiply-adds = 8 int8 ops
PEAK_INT8_OPS = 5.0e15           # MI355X dense int8 MFMA, ops/s (2.4 GHz)
PEAK_HBM_GBS = 8000.0            # MI355X HBM3E, GB/s
CHANNEL_HZ = 24.0e3              # channel width of the paper's F-engine (Section 2)


KERNEL = "xcorr_wg_kernel"        # the dominant kernel of a step
PROFILES = os.path.join(ROOT, "profiles")
# device code the traffic counters depend on (the kernel and the helpers it
# uses); host-only changes elsewhere do not invalidate them
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1411_3751_amd", "csrc", f)
                  for f in ("xcorr_wg.h", "xcorr_i8.h")]
SN_SOURCES = ["xcorr_sn.h", "xcorr_wg.h", "xcorr_i8.h"]  # the small-N kernel and its helpers


def code_text(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed:
    what the compiler sees, so that a comment edit keeps a summary valid."""
    import re
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def kernel_source_hash(files=None) -> str:
    import hashlib
    h = hashlib.sha256()
    srcs = KERNEL_SOURCES if files is None else [
        os.path.join(ROOT, "paper_1411_3751_amd", "csrc", f) for f in files]
    for f in srcs:
        with open(f, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def hbm_traffic(kernel: str, workload: str, files=None):
    """HBM bytes per launch from the committed counter summary, or None.

    The summary holds FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
    kernel on this workload and the same counters for a plain device copy of
    known size; the copy gives the factor that turns counts into bytes. The
    figure is used only while the kernel sources still hash to the value the
    summary was taken from.
    """
    path = os.path.join(PROFILES, "%s.%s.traffic.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash(files):
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(samples, n_inputs, n_chans, n_time, in_bits=4, budget_s=15.0):
    """Time the CPU oracle on a bounded sample of the same gulp (whole channels)."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    tri = n_inputs * (n_inputs + 1) // 2
    cores = oracle.num_threads()
    # calibrate on one channel, then size the sample to about budget_s seconds
    t0 = time.perf_counter()
    oracle.correlate(samples, in_bits, chans=[0])
    one = time.perf_counter() - t0
    n_sel = int(max(1, min(n_chans, round(budget_s / max(one, 1e-3) * cores / 2))))
    n_sel = max(cores, (n_sel // cores) * cores) if n_sel >= cores else n_sel
    n_sel = min(n_sel, n_chans)
    chans = np.linspace(0, n_chans - 1, n_sel).round().astype(int).tolist()
    t0 = time.perf_counter()
    oracle.correlate(samples, in_bits, chans=chans)
    dt = time.perf_counter() - t0
    cmac = n_sel * tri * n_time
    return {"value": cmac * OPS_PER_CMAC / dt / 1e12, "unit": "Tops/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d of %d channels of the same gulp (N=%d, T=%d), %.1f s" % (
                n_sel, n_chans, n_inputs, n_time, dt),
            "cmac_per_s": cmac / dt,
            # the oracle runs one channel per thread: the calibration call
            # above (one channel) ran on one core
            "cmac_per_s_one_core": tri * n_time / one,
            "cpu_model": cpu_model()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


STREAM_CFG = dict(n_inputs=512, n_chans=2400, n_time=8192, in_bits=4)  # 2400 x 24 kHz, 0.341 s gulps


def stream_bench(args):
    """Real-time streaming: a continuous 4-bit stream (drifting common tone)
    produced on the device gulp by gulp into a 4-slot ring, integrated and
    dumped every 26 gulps. Reports sustained Tops/s and real-time factor
    (unpaced), per-gulp latency percentiles (gulps injected at a fixed rate),
    and checks one dump period against the oracle."""
    import numpy as np
    import torch

    import synth
    import synth.gpu
    from paper_1411_3751_amd import Stream

    torch.cuda.set_device(0)
    synth.gpu.build()
    N, F, T = STREAM_CFG["n_inputs"], STREAM_CFG["n_chans"], STREAM_CFG["n_time"]
    every, slots = args.dump_every, 4
    seed = synth.SEED_BASE + 4
    tone = (synth.TONE_AMP, lambda t: synth.drift_phase(t, T), synth.tone_channels(F))
    n_max = max(args.stream_gulps + 8, every)
    gen = synth.gpu.DeviceStream(seed, F, N, 4, 2.5, tone=tone, t_total=n_max * T)
    tri = N * (N + 1) // 2
    cmac_gulp = F * tri * T
    gulp_s = T / CHANNEL_HZ
    hd = [torch.empty((F, tri, 2), dtype=torch.int32, pin_memory=True) for _ in range(2)]
    sub = dict(STREAM_CFG)
    res = {}

    def feed(st, g0, n, pace_s=0.0):
        t_next = time.perf_counter()
        for g in range(g0, g0 + n):
            if pace_s:
                while time.perf_counter() < t_next:
                    time.sleep(0.0005)
                t_next += pace_s
            ptr, ist = st.next_slot()
            gen.fill(ptr, g * T, T, ist)
            st.push()

    # 1. one dump period, checked against the oracle (sampled channels)
    log("stream: verification period (%d gulps) ..." % every)
    with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
        feed(st, 0, every)
        st.dump_wait(0)
        got = hd[0].numpy().copy()
    rng = np.random.default_rng(55)
    tch = synth.tone_channels(F)
    chans = tch + sorted(rng.choice([f for f in range(F) if f not in tch], 4, replace=False).tolist())
    proj = sorted(rng.choice([f for f in range(F) if f not in chans], 8, replace=False).tolist())
    import oracle
    oracle.build(force=False)
    x, _, _ = synth.stream(seed, every * T, F, N, 4, 2.5, chans=chans + proj, tone=tone)
    xs = np.ascontiguousarray(x[:, :len(chans)])
    want = oracle.narrow(oracle.correlate(xs, 4))
    exact = bool(np.array_equal(got[chans], want))
    proj_ok = True
    for k, f in enumerate(proj):
        w = rng.integers(-4, 5, size=(N, 2)).astype(np.int64)
        xp = np.ascontiguousarray(x[:, len(chans) + k:len(chans) + k + 1])
        proj_ok &= oracle.projection_check(xp, 4, 0, got[f], w) == 0
    del x, xs
    res["dump0_exact_channels"] = chans
    res["dump0_exact"] = exact
    res["dump0_projection_channels"] = proj
    res["dump0_projection_ok"] = bool(proj_ok)
    log("stream: dump 0 exact on %d channels: %s, projection on %d: %s" % (
        len(chans), exact, len(proj), proj_ok))

    # 2. unpaced: sustained throughput and real-time factor
    n = args.stream_gulps
    with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
        feed(st, 0, 2 * slots)          # warm-up gulps (not timed)
        st.gulp_times(2 * slots - 1)
        t0 = time.perf_counter()
        feed(st, 2 * slots, n)
        st.gulp_times(2 * slots + n - 1)
        wall = time.perf_counter() - t0
    res["sustained_tops_with_generator"] = cmac_gulp * n * OPS_PER_CMAC / wall / 1e12
    res["rtf_with_generator"] = n * gulp_s / wall
    res["gulps_timed"] = n
    log("stream: %d gulps with the device generator in the loop in %.2f s: %.1f Tops/s, RTF %.1f" % (
        n, wall, res["sustained_tops_with_generator"], res["rtf_with_generator"]))

    # 2b. the ring alone: slots filled once, then every gulp reuses its slot's
    # contents (next_slot / push without refilling), so the sustained rate is
    # that of the X-engine and the ring machinery, not of the test generator
    with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
        feed(st, 0, slots)
        st.gulp_times(slots - 1)
        t0 = time.perf_counter()
        for _ in range(n):
            st.next_slot()
            st.push()
        st.gulp_times(slots + n - 1)
        wall = time.perf_counter() - t0
    res["sustained_tops"] = cmac_gulp * n * OPS_PER_CMAC / wall / 1e12
    res["rtf"] = n * gulp_s / wall
    log("stream: %d gulps through the ring (slots filled once) in %.2f s: %.1f Tops/s, RTF %.1f" % (
        n, wall, res["sustained_tops"], res["rtf"]))

    # 3. paced: gulps arrive every gulp_s / pace seconds; latency percentiles
    pace = args.pace
    with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
        feed(st, 0, n, pace_s=gulp_s / pace)
        lat = [st.gulp_times(g) for g in range(n)]
    arr = np.array([a for a, _ in lat])
    rdy = np.array([r for _, r in lat])
    xe = float(np.percentile(rdy, 50))
    res.update({
        "xengine_gulp_ms_p50": xe,
        "xengine_tops_p50": cmac_gulp * OPS_PER_CMAC / (xe * 1e-3) / 1e12,
        "xengine_rtf_p50": gulp_s / (xe * 1e-3),
        "pace_x_realtime": pace,
        "gulp_ms_p50": float(np.percentile(rdy, 50)), "gulp_ms_p99": float(np.percentile(rdy, 99)),
        "gulp_ms_max": float(rdy.max()),
        "ingest_gulp_ms_p50": float(np.percentile(arr, 50)),
        "ingest_gulp_ms_p99": float(np.percentile(arr, 99)),
    })
    # 4. H2D-inclusive: gulps replayed from a pool of pinned host buffers by
    # hipMemcpyAsync on the ring's ingest stream (PCIe in the loop)
    if args.stream_h2d_gulps > 0:
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        hip.hipHostMalloc.argtypes = [ctypes.POINTER(vp), sz, ctypes.c_uint]
        hip.hipHostFree.argtypes = [vp]
        hip.hipMemcpy.argtypes = [vp, vp, sz, ctypes.c_int]
        hip.hipMemcpyAsync.argtypes = [vp, vp, sz, ctypes.c_int, vp]
        nbytes = F * N * T
        pool = []
        for g in range(2):
            p_ = vp()
            if hip.hipHostMalloc(ctypes.byref(p_), nbytes, 0) != 0:
                raise RuntimeError("hipHostMalloc of %d bytes failed" % nbytes)
            pool.append(p_)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        for g, p_ in enumerate(pool):
            gen.fill(scratch.data_ptr(), g * T, T, torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            if hip.hipMemcpy(p_, scratch.data_ptr(), nbytes, 2) != 0:
                raise RuntimeError("hipMemcpy D2H failed")
        del scratch
        torch.cuda.empty_cache()
        nh = args.stream_h2d_gulps

        def feed_h2d(st, g0, cnt):
            for g in range(g0, g0 + cnt):
                ptr, ist = st.next_slot()
                if hip.hipMemcpyAsync(ptr, pool[g % 2], nbytes, 1, ist) != 0:
                    raise RuntimeError("hipMemcpyAsync H2D failed")
                st.push()

        with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
            feed_h2d(st, 0, slots)
            st.gulp_times(slots - 1)
            t0 = time.perf_counter()
            feed_h2d(st, slots, nh)
            st.gulp_times(slots + nh - 1)
            wall = time.perf_counter() - t0
        for p_ in pool:
            hip.hipHostFree(p_)
        res["rtf_h2d"] = nh * gulp_s / wall
        res["h2d_gbs"] = nh * nbytes / wall / 1e9
        res["gulps_timed_h2d"] = nh
        log("stream: H2D-inclusive %d gulps in %.2f s: RTF %.2f, %.1f GB/s" % (
            nh, wall, res["rtf_h2d"], res["h2d_gbs"]))

    out = {
        "metric": METRIC, "value": round(res["sustained_tops"], 2), "unit": "Tops/s",
        "n_gpus": 1, "steps": n, "warmup": 2 * slots, "ms_per_step": round(1e3 * gulp_s / res["rtf"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "stream_2400ch", "n_inputs": N, "n_chans": F, "n_time": T,
                   "in_bits": 4, "engine": "i8", "ring_slots": slots, "dump_every": every,
                   "ingest": "device generator (counter-based, drifting tone) for the checked "
                             "period, the latency run and the *_with_generator figures; slots "
                             "filled once for value/rtf"},
    }
    out.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in res.items()})
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Batched subarrays of uneven N (64 ... 2048 inputs, 4096 samples each):
    autotuned kernel choices, one persistent launch per engine and input
    width, the whole step (correlate + dump) captured in a HIP graph and
    replayed."""
    import torch

    import synth
    from paper_1411_3751_amd import Correlator

    torch.cuda.set_device(0)
    subs, dev, cmac = [], [], 0
    for k in range(len(synth.BATCH_SHAPES)):
        x, _, _, meta = synth.workload("batch", subarray=k)
        N, F, T = meta["n_inputs"], meta["n_chans"], meta["n_time"]
        subs.append(dict(n_inputs=N, n_chans=F, n_time=T))
        dev.append(torch.from_numpy(x).cuda())
        cmac += F * N * (N + 1) // 2 * T
    out = [torch.empty((d["n_chans"], d["n_inputs"] * (d["n_inputs"] + 1) // 2, 2),
                       dtype=torch.int32, device="cuda") for d in subs]
    stream = torch.cuda.current_stream()
    with Correlator(subs, stream=stream) as c:
        t0 = time.perf_counter()
        c.autotune(dev, reps=5)
        tune_s = time.perf_counter() - t0
        plan = c.plan()
        log("plan:", json.dumps(plan))
        with c.capture(dev, out) as g:
            for _ in range(args.warmup):
                g.launch(stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                g.launch(stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
    value = cmac * OPS_PER_CMAC / (ms * 1e-3) / 1e12
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Tops/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "batch_uneven", "subarrays": [[d["n_inputs"], d["n_chans"]] for d in subs],
                   "n_time": subs[0]["n_time"], "in_bits": 4, "engine": "i8",
                   "step": "graph replay: correlate + dump"},
        "pct_int8_peak": round(100.0 * value / (PEAK_INT8_OPS / 1e12), 2),
        "autotune_s": round(tune_s, 2),
        "choices": [[s["n_inputs"], s["kernel"], s.get("tile")] for s in plan["subarrays"]],
        "schedule": [plan["workgroups_per_cu"], plan["schedule_order"]],
    }
    print(json.dumps(res), flush=True)


def sweep_bench(args):
    """The X-engine across N at T = 8192 (4-bit, int8 engine, the headline's
    step: correlate + dump in one xeng_correlate_dump call, default plan), F
    chosen so each shape does comparable work; one JSON line whose value is
    the N = 512 shape."""
    import torch

    from paper_1411_3751_amd import Correlator

    torch.cuda.set_device(0)
    T = 8192
    shapes = [(128, 1024), (256, 512), (512, 128), (768, 96), (1024, 64), (2048, 16), (4096, 4)]
    rows = []
    g = torch.Generator(device="cuda").manual_seed(11)
    for N, F in shapes:
        x = torch.randint(0, 256, (T, F, N), dtype=torch.int32, device="cuda", generator=g).to(torch.uint8)
        out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
        with Correlator([dict(n_inputs=N, n_chans=F, n_time=T)]) as c:
            kern = c.plan()["subarrays"][0]["kernel"]
            for _ in range(args.warmup):
                c.correlate_dump([x], [out])
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                c.correlate_dump([x], [out])
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
        del x, out
        ops = F * N * (N + 1) // 2 * T * OPS_PER_CMAC
        nb = (N + 127) // 128
        computed = (nb * (nb + 1) // 2 - nb) * 16384 + nb * 10240  # cells per channel
        rows.append({"n_inputs": N, "n_chans": F, "kernel": kern, "ms": round(ms, 4),
                     "tops": round(ops / (ms * 1e-3) / 1e12, 1),
                     "pct_int8_peak": round(100.0 * ops / (ms * 1e-3) / PEAK_INT8_OPS, 2),
                     "useful_fraction": round(N * (N + 1) / 2 / computed, 3)})
        log("N=%d F=%d %s %.4f ms" % (N, F, kern, ms))
    main_row = [r for r in rows if r["n_inputs"] == 512][0]
    res = {"metric": METRIC, "value": main_row["tops"], "unit": "Tops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_row["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
           "data": "synthetic",
           "config": {"workload": "sweep_n", "n_time": T, "in_bits": 4, "engine": "i8",
                      "step": "correlate + dump (device, reset) in one xeng_correlate_dump call",
                      "value_of": "N=512, F=128"},
           "sweep": rows}
    print(json.dumps(res), flush=True)


def ingest_bench(args):
    """Packet ingest: the LEDA gulp (N=512, 128 channels, 8192 samples) cut
    into F-engine packets of 4 times x 16 channels x 64 inputs (4 KB payload),
    5 % lost and shuffled; the corner turn into the gulp is timed (HBM-bound:
    bytes = packets read + gulp written)."""
    import numpy as np
    import torch

    import synth
    from paper_1411_3751_amd import Ingest

    torch.cuda.set_device(0)
    samples, _, _, meta = synth.workload("leda_gulp")
    N, F, T = meta["n_inputs"], meta["n_chans"], meta["n_time"]
    fmt = (4, 16, 64)
    t0 = 5 * T
    pk = synth.packetize(samples, t0, *fmt)
    rng = np.random.default_rng(3)
    pk = np.ascontiguousarray(pk[rng.permutation(len(pk))[: int(0.95 * len(pk))]])
    d_pk = torch.from_numpy(pk.reshape(-1)).cuda()
    gulp = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    with Ingest(dict(n_inputs=N, n_chans=F, n_time=T), *fmt) as ig:
        for _ in range(args.warmup):
            ig.gulp(d_pk, len(pk), t0, gulp, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            ig.gulp(d_pk, len(pk), t0, gulp, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        st = ig.stats()
    nbytes = pk.nbytes + gulp.numel()
    res = {"metric": "packet ingest (corner turn) GB/s", "value": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "leda_gulp_packets", "n_inputs": N, "n_chans": F, "n_time": T,
                      "packet": list(fmt), "packets": len(pk), "lost_fraction": 0.05},
           "packets_per_s": round(len(pk) / (ms * 1e-3)), "stats": st,
           "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 1),
                        "peak": 8000.0, "unit": "GB/s",
                        "frac": round(nbytes / (ms * 1e-3) / 8e12, 4), "traffic": None}}
    print(json.dumps(res), flush=True)


FENGINE_CFG = dict(n_inputs=512, chan0=1250, n_chans=2398, n_spectra=64, gain=22.0, seed=7)
ADC_HZ = 196.608e6               # the paper's ADC sample clock (Section 2.2)
FE_P, FE_TAPS = 8192, 4
# algorithmic operations per spectrum of one input: the FIR's multiply-adds
# (2 taps P) plus the usual 2.5 P log2 P flops of a P-point real FFT
FE_OPS_PER_SPECTRUM = 2 * FE_TAPS * FE_P + 2.5 * FE_P * 13
PEAK_FP32_VECTOR = 157.3e12      # MI355X vector fp32, flop/s


def fengine_cpu_baseline(adc_rows, gain, chan0, n_chans, budget_s=12.0):
    """The reference F-engine on a bounded sample: whole spectra of a few inputs."""
    from oracle import fengine as fe
    n_rows, S = adc_rows.shape
    n_m = S // FE_P - (FE_TAPS - 1)
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < budget_s:
        m = done % n_m
        fe.fengine(adc_rows, 0, gain, chan0, n_chans, spectra=[m])
        done += 1
    dt = time.perf_counter() - t0
    samples = done * n_rows * FE_P
    return {"value": round(samples / dt / 1e9, 4), "unit": "Gsamples/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d spectra of %d inputs (%d ADC samples each), %.1f s" % (
                done, n_rows, FE_P, dt)}


def fengine_bench(args):
    """F-engine: 512 ADC inputs, 64 spectra per call (8192 new samples each),
    PFB + FFT + requantisation of channels 1250..3647 (30-88 MHz) into the
    X-engine's 4+4-bit layout. Input resident in HBM; each call is one launch."""
    import torch

    import synth
    from paper_1411_3751_amd import FEngine

    torch.cuda.set_device(0)
    c = FENGINE_CFG
    N, M, F = c["n_inputs"], c["n_spectra"], c["n_chans"]
    S = FE_P * (M + FE_TAPS - 1)
    log("generating %d x %d ADC samples on the device ..." % (N, S))
    d_adc = synth.adc_device(c["seed"], N, S, "cuda")
    out = torch.empty((M, F, N), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    with FEngine(N, c["chan0"], F, c["gain"]) as f:
        for _ in range(args.warmup):
            f.run(d_adc, M, out, stream=stream)
        torch.cuda.synchronize()
        n = args.steps
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        k_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(n)]
        t_start.record(stream)
        for k in range(n):
            k_ev[k][0].record(stream)
            f.run(d_adc, M, out, stream=stream)
            k_ev[k][1].record(stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        group = f.group
    ms_step = t_start.elapsed_time(t_end) / n
    ms_kernel = sum(a.elapsed_time(b) for a, b in k_ev) / n
    samples = N * M * FE_P
    value = samples / (ms_step * 1e-3)
    ops = N * M * FE_OPS_PER_SPECTRUM
    achieved = ops / (ms_kernel * 1e-3)
    res = {"metric": "F-engine ADC samples/s (Gsamples/s) at N=512; real-time factor at 196.608 MS/s",
           "value": round(value / 1e9, 2), "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "fengine_512", "n_inputs": N, "n_spectra": M,
                      "chan0": c["chan0"], "n_chans": F, "fft": FE_P, "taps": FE_TAPS,
                      "gain": c["gain"], "group": group},
           "rtf": round(value / (N * ADC_HZ), 2),
           "spectra_per_s": round(N * M / (ms_step * 1e-3)),
           "ms_kernel": round(ms_kernel, 4),
           "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 2),
                        "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP32_VECTOR, 4),
                        "traffic": hbm_traffic("fengine_kernel", "fengine_512",
                                               ["xeng_fengine.h"])}}
    if not args.no_cpu:
        log("timing the CPU reference F-engine on a sample ...")
        rows = d_adc[:4, :FE_P * (FE_TAPS + 3)].cpu().numpy()
        res["cpu_baseline"] = fengine_cpu_baseline(rows, c["gain"], c["chan0"], F)
    print(json.dumps(res), flush=True)


def fx_bench(args):
    """The whole FX correlator on one GPU: per 8192-sample gulp, the F-engine
    channelises 512 ADC inputs (64 spectra per launch, channels 1250..3647)
    straight into the gulp buffer, then the X-engine integrates the gulp.
    The ADC block of one launch is reused for every launch (contents do not
    change the work). Reports ms per gulp and the real-time factor."""
    import torch

    import synth
    from paper_1411_3751_amd import Correlator, FEngine

    torch.cuda.set_device(0)
    c = FENGINE_CFG
    N, M, F, T = c["n_inputs"], c["n_spectra"], c["n_chans"], 8192
    S = FE_P * (M + FE_TAPS - 1)
    log("generating %d x %d ADC samples on the device ..." % (N, S))
    d_adc = synth.adc_device(c["seed"], N, S, "cuda")
    gulp = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    fe = FEngine(N, c["chan0"], F, c["gain"])
    xc = Correlator([dict(n_inputs=N, n_chans=F, n_time=T, in_bits=4)], stream=stream)

    def one_gulp():
        for m0 in range(0, T, M):
            fe.run(d_adc, M, gulp[m0:m0 + M], stream=stream)
        xc.correlate([gulp])

    for _ in range(max(1, args.warmup)):
        one_gulp()
    xc.reset()
    torch.cuda.synchronize()
    n = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n)]
    for g in range(n):
        ev[g][0].record(stream)
        for m0 in range(0, T, M):
            fe.run(d_adc, M, gulp[m0:m0 + M], stream=stream)
        ev[g][1].record(stream)
        xc.correlate([gulp])
        ev[g][2].record(stream)
    torch.cuda.synchronize()
    ms = ev[0][0].elapsed_time(ev[-1][2]) / n
    ms_f = sum(a.elapsed_time(b) for a, b, _ in ev) / n
    ms_x = sum(b.elapsed_time(c) for _, b, c in ev) / n
    out = xc.dump()[0]
    torch.cuda.synchronize()
    xc.close()
    fe.close()
    gulp_s = T / CHANNEL_HZ
    tri = N * (N + 1) // 2
    res = {"metric": "end-to-end FX correlator real-time factor at N=512 (F-engine + X-engine per gulp)",
           "value": round(gulp_s / (ms * 1e-3), 2), "unit": "x real time", "n_gpus": 1, "steps": n,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+int8", "data": "synthetic",
           "config": {"workload": "fx_512", "n_inputs": N, "n_chans": F, "n_time": T,
                      "chan0": c["chan0"], "fft": FE_P, "taps": FE_TAPS, "gain": c["gain"]},
           "ms_fengine": round(ms_f, 3), "ms_xengine": round(ms_x, 3),
           "fengine_gsamples_per_s": round(N * T * FE_P / (ms_f * 1e-3) / 1e9, 1),
           "xengine_tops": round(F * tri * T * OPS_PER_CMAC / (ms_x * 1e-3) / 1e12, 1),
           "dump_shape": list(out.shape)}
    print(json.dumps(res), flush=True)


def fx_stream_bench(args):
    """The FX correlator as a real-time pipeline: for each 8192-sample gulp the
    F-engine channelises the 512 ADC inputs (2398 channels) into the next slot
    of the X-engine's 4-slot device ring on the ring's ingest stream, and the
    X-engine integrates it on its compute stream, dumping every 26 gulps; the
    F-engine of one gulp overlaps the X-engine of the one before. Reports the
    sustained real-time factor and per-gulp latency percentiles."""
    import numpy as np
    import torch

    import synth
    from paper_1411_3751_amd import FEngine, Stream

    torch.cuda.set_device(0)
    c = FENGINE_CFG
    N, M, F, T = c["n_inputs"], c["n_spectra"], c["n_chans"], 8192
    S = FE_P * (M + FE_TAPS - 1)
    log("generating %d x %d ADC samples on the device ..." % (N, S))
    d_adc = synth.adc_device(c["seed"], N, S, "cuda")
    torch.cuda.synchronize()
    fe = FEngine(N, c["chan0"], F, c["gain"])
    sub = dict(n_inputs=N, n_chans=F, n_time=T, in_bits=4)
    slots, every = 4, args.dump_every
    gulp_s = T / CHANNEL_HZ

    def feed(st, cnt):
        for _ in range(cnt):
            ptr, ist = st.next_slot()
            for m0 in range(0, T, M):
                fe.run_ptr(d_adc.data_ptr(), S, M, ptr + m0 * F * N, 0, ist)
            st.push()

    n = args.steps
    with Stream(sub, n_slots=slots, dump_every=every) as st:
        feed(st, slots)
        st.gulp_times(slots - 1)
        t0 = time.perf_counter()
        feed(st, n)
        st.gulp_times(slots + n - 1)
        wall = time.perf_counter() - t0
        lat = [st.gulp_times(g) for g in range(slots, slots + n)]
    fe.close()
    rdy = np.array([r for _, r in lat])
    arr = np.array([a for a, _ in lat])
    rtf = n * gulp_s / wall
    res = {"metric": "FX correlator streaming real-time factor at N=512 (F-engine into the X-engine ring)",
           "value": round(rtf, 2), "unit": "x real time", "n_gpus": 1, "steps": n,
           "warmup": slots, "ms_per_step": round(1e3 * wall / n, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+int8", "data": "synthetic",
           "config": {"workload": "fx_stream_512", "n_inputs": N, "n_chans": F, "n_time": T,
                      "ring_slots": slots, "dump_every": every, "chan0": c["chan0"],
                      "fft": FE_P, "taps": FE_TAPS, "gain": c["gain"]},
           "gulp_ms_p50": round(float(np.percentile(rdy, 50)), 3),
           "gulp_ms_p99": round(float(np.percentile(rdy, 99)), 3),
           "arrival_to_done_ms_p50": round(float(np.percentile(arr, 50)), 3),
           "arrival_to_done_ms_p99": round(float(np.percentile(arr, 99)), 3)}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--workload", default="leda_gulp",
                    choices=["leda_gulp", "fp8_variant", "int8_variant", "tiny", "n64"],
                    help="input shape (the default is the headline configuration; fp8_variant and "
                         "int8_variant time the precision variants; tiny (N=32) and n64 (N=64, "
                         "512 channels, 4096 samples) the small-N, memory-bound regime)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its kernel and schedule choices on the input first")
    ap.add_argument("--engine", default=None, choices=["i8", "fp8"],
                    help="arithmetic engine (default: fp8 for fp8_variant, else i8)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times), the "
                         "reference for scaling HBM byte counters, and exit")
    ap.add_argument("--stream", action="store_true",
                    help="run the real-time streaming configuration instead (N=512, 2400 "
                         "channels, 8192-sample gulps, 4-slot ring)")
    ap.add_argument("--batch", action="store_true",
                    help="run the batched uneven-subarray configuration instead (autotuned, "
                         "graph-captured)")
    ap.add_argument("--sweep", action="store_true",
                    help="time the X-engine alone across N = 128 ... 4096 at T = 8192")
    ap.add_argument("--ingest", action="store_true",
                    help="time the packet ingest (corner turn of F-engine packets) instead")
    ap.add_argument("--fengine", action="store_true",
                    help="time the F-engine (PFB + FFT + 4+4-bit requantisation) instead")
    ap.add_argument("--fx", action="store_true",
                    help="time F-engine + X-engine per 8192-sample gulp (512 inputs, 2398 channels)")
    ap.add_argument("--fx-stream", action="store_true",
                    help="the same as a pipeline through the X-engine's streaming ring")
    ap.add_argument("--stream-gulps", type=int, default=260)
    ap.add_argument("--stream-h2d-gulps", type=int, default=12,
                    help="stream mode: gulps timed with the input copied from pinned host memory "
                         "(0 skips that phase)")
    ap.add_argument("--dump-every", type=int, default=26)
    ap.add_argument("--pace", type=float, default=10.0,
                    help="latency run: gulps arrive at this multiple of the real-time rate")
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed back-to-back steps before the warm-up steps")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streaming figures of the default line")
    args = ap.parse_args()
    if args.fx_stream:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        fx_stream_bench(args)
        return
    if args.fx:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        fx_bench(args)
        return
    if args.fengine:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        fengine_bench(args)
        return
    if args.sweep:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        sweep_bench(args)
        return
    if args.ingest:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        ingest_bench(args)
        return
    if args.batch:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        batch_bench(args)
        return
    if args.stream:
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus %d requested)" % args.gpus, file=sys.stderr)
            sys.exit(2)
        stream_bench(args)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path (--gpus %d "
              "requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    xengine_bench(args)


def xengine_bench(args):
    """The headline step on one workload: xeng_correlate + xeng_dump(device,
    reset) with the samples resident in HBM."""
    import torch

    import synth
    from paper_1411_3751_amd import Correlator

    torch.cuda.set_device(0)
    name = args.workload
    engine = args.engine or ("fp8" if name == "fp8_variant" else "i8")
    log("generating workload %s ..." % name)
    samples, _, _, meta = synth.workload(name)
    N, F, T = meta["n_inputs"], meta["n_chans"], meta["n_time"]
    in_bits = meta["in_bits"]
    tri = N * (N + 1) // 2
    cmac_per_step = F * tri * T
    d_samples = torch.from_numpy(samples).cuda()
    out = torch.empty((F, tri, 2), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    corr = Correlator([dict(n_inputs=N, n_chans=F, n_time=T, in_bits=in_bits,
                            engine=1 if engine == "fp8" else 0)], stream=stream)
    if args.autotune:
        corr.autotune([d_samples])
    plan = corr.plan()
    log("plan:", json.dumps(plan))

    def step():
        corr.correlate_dump([d_samples], [out])

    # settle: under sustained MFMA load the clock first overshoots downwards
    # and recovers over the next tens of milliseconds; a fixed stretch of
    # untimed steps puts the warm-up and the timed steps in the settled state
    settle_steps = settle(step, args.settle_s)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps between two events, nothing else enqueued
    n = args.steps
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(n):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_step = t_start.elapsed_time(t_end) / n
    # clock under the same load, read between batches of queued steps (not
    # during the timed region: the readings take host time)
    mhz = clock_under_load(step, max(8, int(12.0 / max(ms_step, 1e-3))))

    # kernel pass (after the timed region): an event pair on the stream
    # around each launch of the tile kernel. With a tile kernel that fuses the
    # dump and at most 32768 samples the step is that one launch; otherwise
    # the pair brackets the correlate call and the dump runs outside it
    k_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(n)]
    fused = plan["subarrays"][0]["kernel"] != "register_staging" and T <= 32768
    for k in range(n):
        k_ev[k][0].record(stream)
        if fused:
            corr.correlate_dump([d_samples], [out])
        else:
            corr.correlate([d_samples])
        k_ev[k][1].record(stream)
        if not fused:
            corr.dump([out], reset=True)
    torch.cuda.synchronize()
    k_ms = [a.elapsed_time(b) for a, b in k_ev]
    ms_kernel = sum(k_ms) / n
    corr.close()
    del d_samples, out
    torch.cuda.empty_cache()

    ops_step = cmac_per_step * OPS_PER_CMAC
    value = ops_step / (ms_step * 1e-3) / 1e12
    achieved = ops_step / (ms_kernel * 1e-3) / 1e12
    peak = PEAK_INT8_OPS / 1e12
    small = N < 256  # tiny and n64: the samples and the output, not the MFMAs, bound the step
    hbm_bytes = N * F * T * (in_bits // 4) + F * tri * 8
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Tops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8_e4m3" if engine == "fp8" else "int8",
        "data": "synthetic",
        "config": {"workload": name, "n_inputs": N, "n_chans": F, "n_time": T,
                   "in_bits": in_bits, "engine": engine, "autotuned": bool(args.autotune),
                   "step": "correlate + dump (device, reset) in one xeng_correlate_dump call",
                   "kernel": plan["subarrays"][0]["kernel"]},
        "settle_steps": settle_steps,
        "settle_s": args.settle_s,
        "cmac_per_s": cmac_per_step / (ms_step * 1e-3),
        "pct_int8_peak": round(100.0 * value / peak, 2),
        # one gulp of this workload (T samples at 24 kHz per channel) against its step time
        "rtf_this_gulp": round(T / CHANNEL_HZ / (ms_step * 1e-3), 1),
        "rtf_this_gulp_def": "%d-sample gulp of %d channels (%.3f s of stream) / step time" % (
            T, F, T / CHANNEL_HZ),
        # minimum HBM bytes of a step: the samples once plus the visibilities once
        "hbm_gbs_algorithmic": round(hbm_bytes / (ms_step * 1e-3) / 1e9, 1),
        "ms_kernel": round(ms_kernel, 4),
        "ms_kernel_p50": round(sorted(k_ms)[n // 2], 4),
    }
    if mhz:
        res["gfxclk_mhz"] = round(mhz, 0)
        res["pct_int8_peak_at_measured_clock"] = round(
            100.0 * value / (PEAK_INT8_OPS * mhz / 2400.0 / 1e12), 2)
        res["clock_source"] = ("amdsmi gpu_metrics current_gfxclks, mean over XCDs, median of "
                               "readings between batches of the same steps after the timed region")
    if small:
        sn = plan["subarrays"][0]["kernel"] == "small_n"
        res["roofline"] = {"bound": "hbm", "achieved": round(hbm_bytes / (ms_kernel * 1e-3) / 1e9, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(hbm_bytes / (ms_kernel * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                           "traffic": hbm_traffic("xcorr_sn_kernel", name, SN_SOURCES) if sn else None}
    else:
        res["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                           "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                           "traffic": hbm_traffic(KERNEL, name) if engine == "i8" and in_bits == 4
                           else None}
    if name == "leda_gulp" and not args.no_stream:
        res.update(stream_figures(args))
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        res["cpu_baseline"] = cpu_baseline(samples, N, F, T, in_bits)
    print(json.dumps(res), flush=True)


def settle(step, seconds):
    """Run back-to-back untimed steps for about `seconds`; returns the count."""
    import torch
    if seconds <= 0:
        return 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            step()
        n += 10
        torch.cuda.synchronize()
    return n


def clock_under_load(step, per_batch, batches=12):
    """Median graphics clock (MHz, mean over the XCDs) read from amdsmi GPU
    metrics between batches of `per_batch` queued steps, or None where the
    metrics are not readable. Each reading is taken while the previous batch
    still runs on the device."""
    import statistics

    import torch
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        h = amdsmi.amdsmi_get_processor_handles()[0]
    except Exception as e:  # no amdsmi, no device, no permission
        log("clock readings unavailable: %s" % e)
        return None
    vals = []
    for b in range(batches):
        for _ in range(per_batch):
            step()
        if b < 2:
            continue  # the metrics table lags the load
        try:
            m = amdsmi.amdsmi_get_gpu_metrics_info(h)
            xs = [float(x) for x in m.get("current_gfxclks", []) if isinstance(x, (int, float))
                  and 0 < x < 10000]
            if xs:
                vals.append(sum(xs) / len(xs))
        except Exception:
            pass
    torch.cuda.synchronize()
    return statistics.median(vals) if vals else None


def stream_figures(args):
    """Real-time figures of the streaming configuration (N = 512, 2400
    channels of 24 kHz, 8192-sample gulps into a 4-slot device ring, dump
    every 26 gulps copied to pinned host buffers): the sustained rate through
    the ring with the slots filled once by the device generator (samples
    resident in HBM, like the step above), and the arrival-to-done latency of
    gulps fed at a fixed multiple of the real-time rate."""
    import numpy as np
    import torch

    import synth
    import synth.gpu
    from paper_1411_3751_amd import Stream

    synth.gpu.build()
    N, F, T = STREAM_CFG["n_inputs"], STREAM_CFG["n_chans"], STREAM_CFG["n_time"]
    every, slots, n = args.dump_every, 4, args.stream_gulps
    seed = synth.SEED_BASE + 4
    tone = (synth.TONE_AMP, lambda t: synth.drift_phase(t, T), synth.tone_channels(F))
    gen = synth.gpu.DeviceStream(seed, F, N, 4, 2.5, tone=tone, t_total=slots * T)
    tri = N * (N + 1) // 2
    cmac_gulp = F * tri * T
    gulp_s = T / CHANNEL_HZ
    hd = [torch.empty((F, tri, 2), dtype=torch.int32, pin_memory=True) for _ in range(2)]
    sub = dict(STREAM_CFG)
    log("stream figures: N=%d F=%d T=%d, %d gulps ..." % (N, F, T, n))
    res = {}
    with Stream(sub, n_slots=slots, dump_every=every, host_dumps=hd) as st:
        for g in range(slots):
            ptr, ist = st.next_slot()
            gen.fill(ptr, g * T, T, ist)
            st.push()
        st.gulp_times(slots - 1)
        # sustained: every gulp reuses its slot's contents, as fast as it goes
        t0 = time.perf_counter()
        for _ in range(n):
            st.next_slot()
            st.push()
        st.gulp_times(slots + n - 1)
        wall = time.perf_counter() - t0
        res["stream_rtf"] = round(n * gulp_s / wall, 2)
        res["stream_tops"] = round(cmac_gulp * n * OPS_PER_CMAC / wall / 1e12, 1)
        res["stream_pct_int8_peak"] = round(100.0 * cmac_gulp * n * OPS_PER_CMAC / wall / PEAK_INT8_OPS, 2)
        # paced: a gulp arrives every gulp_s / pace seconds (host clock);
        # latency = arrival (next_slot) to the end of its correlation (and of
        # its dump when it completes one)
        g0 = slots + n
        pace = args.pace
        t_next = time.perf_counter()
        for _ in range(n):
            while time.perf_counter() < t_next:
                time.sleep(0.0002)
            t_next += gulp_s / pace
            st.next_slot()
            st.push()
        lat = np.array([st.gulp_times(g)[0] for g in range(g0, g0 + n)])
    res["stream_gulp_ms_p50"] = round(float(np.percentile(lat, 50)), 3)
    res["stream_gulp_ms_p99"] = round(float(np.percentile(lat, 99)), 3)
    res["stream_gulp_ms_max"] = round(float(lat.max()), 3)
    res["stream_config"] = {"workload": "stream_2400ch", "n_inputs": N, "n_chans": F, "n_time": T,
                            "ring_slots": slots, "dump_every": every, "gulps": n,
                            "pace_x_realtime": pace,
                            "rtf_def": "%d gulps x %.3f s of stream / wall time, slots filled "
                                       "once (samples resident in HBM), dumps copied to pinned "
                                       "host memory" % (n, gulp_s)}
    log("stream figures: RTF %.1f, %.1f Tops/s, latency p50 %.2f ms p99 %.2f ms" % (
        res["stream_rtf"], res["stream_tops"], res["stream_gulp_ms_p50"], res["stream_gulp_ms_p99"]))
    del hd
    return res


if __name__ == "__main__":
    main()
