"""Thin ctypes binding of libxeng.so (include/xeng.h).

Argument marshalling only: every step of the correlation runs in the HIP
library. PyTorch supplies device memory (tensors) and streams. If the built
library is missing this module raises at load time; there is no fallback.
"""
from __future__ import annotations

import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxeng.so")

XENG_OK, XENG_EINVAL, XENG_ERANGE, XENG_ENOMEM, XENG_EHIP, XENG_EBUSY = 0, 1, 2, 3, 4, 5
KERNEL_REGISTER, KERNEL_PERSISTENT, KERNEL_ONE_WAVE, KERNEL_TWO_WAVE, KERNEL_SMALL_N = 0, 1, 2, 3, 4
ENGINE_I8, ENGINE_FP8 = 0, 1
MAX_DUMP_SAMPLES_4BIT = 16777215
MAX_DUMP_SAMPLES_8BIT = 65535
MAX_CALL_SAMPLES_FP8 = 32768

EXPORTS = (
    "xeng_create", "xeng_correlate", "xeng_dump", "xeng_correlate_dump", "xeng_destroy",
    "xeng_correlate_dump_static",
    "xeng_set_stream",
    "xeng_samples_since_dump", "xeng_max_dump_samples", "xeng_plan_describe", "xeng_set_kernel",
    "xeng_strerror", "xeng_last_error",
    "xeng_stream_create", "xeng_stream_next_slot", "xeng_stream_push", "xeng_stream_dump_wait",
    "xeng_stream_gulp_times", "xeng_stream_gulps", "xeng_stream_backlog", "xeng_stream_destroy",
    "xeng_stream_drop", "xeng_stream_set_nonblocking", "xeng_stream_stats",
    "xeng_stream_set_fast_autos", "xeng_stream_fast_wait",
    "xeng_autotune", "xeng_graph_create", "xeng_graph_launch", "xeng_graph_destroy",
    "xeng_tuning_save", "xeng_tuning_load", "xeng_tuning_clear",
    "xeng_set_fast_autos", "xeng_dump_fast_autos",
    "xeng_ingest_create", "xeng_ingest_packet_stride", "xeng_ingest_gulp", "xeng_ingest_stats_get",
    "xeng_ingest_destroy",
    "xeng_fengine_create", "xeng_fengine_group", "xeng_fengine_run", "xeng_fengine_destroy",
)
FENGINE_FFT = 8192
FENGINE_TAPS = 4
FENGINE_CHANS = 4096
PACKET_MAGIC = 0x4C454441


class XengError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("xeng error %d: %s" % (code, msg))
        self.code = code


class PacketFormat(ctypes.Structure):
    _fields_ = [("pkt_time", ctypes.c_int32), ("pkt_chans", ctypes.c_int32),
                ("pkt_inputs", ctypes.c_int32)]


class IngestStats(ctypes.Structure):
    _fields_ = [("received", ctypes.c_int64), ("missing", ctypes.c_int64),
                ("duplicate", ctypes.c_int64), ("rejected", ctypes.c_int64)]


class FEngineConfig(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("chan0", ctypes.c_int32),
                ("n_chans", ctypes.c_int32), ("gain", ctypes.c_float)]


class Subarray(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_chans", ctypes.c_int32),
                ("n_time", ctypes.c_int32), ("in_bits", ctypes.c_int32),
                ("engine", ctypes.c_int32)]


_lib = None


class StreamStats(ctypes.Structure):
    _fields_ = [("gulps", ctypes.c_int64), ("correlated", ctypes.c_int64),
                ("dropped", ctypes.c_int64), ("dumps", ctypes.c_int64),
                ("fast_dumps", ctypes.c_int64), ("backlog", ctypes.c_int64)]


def load():
    """Load libxeng.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libxeng.so is not built (%s); run python -m paper_1411_3751_amd.build"
                          % LIB_PATH)
    # PyTorch first: libxeng.so and torch then share the HIP runtime torch
    # loads (the same soname); loaded the other way round, torch would run on
    # the one libxeng.so found first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.xeng_create.argtypes = [ctypes.POINTER(Subarray), i32, vp, ctypes.POINTER(vp)]
    lib.xeng_create.restype = i32
    lib.xeng_correlate.argtypes = [vp, pp]
    lib.xeng_correlate.restype = i32
    lib.xeng_dump.argtypes = [vp, pp, i32, i32]
    lib.xeng_dump.restype = i32
    lib.xeng_correlate_dump.argtypes = [vp, pp, pp, i32, i32]
    lib.xeng_correlate_dump.restype = i32
    lib.xeng_correlate_dump_static.argtypes = [ctypes.POINTER(Subarray), vp, vp, vp]
    lib.xeng_correlate_dump_static.restype = i32
    lib.xeng_destroy.argtypes = [vp]
    lib.xeng_destroy.restype = i32
    lib.xeng_set_stream.argtypes = [vp, vp]
    lib.xeng_set_stream.restype = i32
    lib.xeng_samples_since_dump.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.xeng_samples_since_dump.restype = i32
    lib.xeng_max_dump_samples.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.xeng_max_dump_samples.restype = i32
    lib.xeng_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.xeng_plan_describe.restype = i32
    lib.xeng_set_kernel.argtypes = [vp, i32, i32, i32]
    lib.xeng_set_kernel.restype = i32
    lib.xeng_strerror.argtypes = [i32]
    lib.xeng_strerror.restype = ctypes.c_char_p
    lib.xeng_last_error.argtypes = []
    lib.xeng_last_error.restype = ctypes.c_char_p
    lib.xeng_stream_create.argtypes = [ctypes.POINTER(Subarray), i32, i32, pp, i32,
                                       ctypes.POINTER(vp)]
    lib.xeng_stream_create.restype = i32
    lib.xeng_stream_next_slot.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.xeng_stream_next_slot.restype = i32
    lib.xeng_stream_push.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xeng_stream_push.restype = i32
    lib.xeng_stream_dump_wait.argtypes = [vp, i64, ctypes.POINTER(vp)]
    lib.xeng_stream_dump_wait.restype = i32
    lib.xeng_stream_gulp_times.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_float)]
    lib.xeng_stream_gulp_times.restype = i32
    lib.xeng_stream_gulps.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xeng_stream_gulps.restype = i32
    lib.xeng_stream_backlog.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xeng_stream_backlog.restype = i32
    lib.xeng_stream_drop.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xeng_stream_drop.restype = i32
    lib.xeng_stream_set_nonblocking.argtypes = [vp, i32]
    lib.xeng_stream_set_nonblocking.restype = i32
    lib.xeng_stream_stats.argtypes = [vp, ctypes.POINTER(StreamStats)]
    lib.xeng_stream_stats.restype = i32
    lib.xeng_stream_set_fast_autos.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32, i32, pp, i32]
    lib.xeng_stream_set_fast_autos.restype = i32
    lib.xeng_stream_fast_wait.argtypes = [vp, i64, ctypes.POINTER(vp)]
    lib.xeng_stream_fast_wait.restype = i32
    lib.xeng_stream_destroy.argtypes = [vp]
    lib.xeng_stream_destroy.restype = i32
    lib.xeng_ingest_create.argtypes = [ctypes.POINTER(Subarray), ctypes.POINTER(PacketFormat),
                                       ctypes.POINTER(vp)]
    lib.xeng_ingest_create.restype = i32
    lib.xeng_ingest_packet_stride.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xeng_ingest_packet_stride.restype = i32
    lib.xeng_ingest_gulp.argtypes = [vp, vp, i64, i64, vp, vp]
    lib.xeng_ingest_gulp.restype = i32
    lib.xeng_ingest_stats_get.argtypes = [vp, ctypes.POINTER(IngestStats)]
    lib.xeng_ingest_stats_get.restype = i32
    lib.xeng_ingest_destroy.argtypes = [vp]
    lib.xeng_ingest_destroy.restype = i32
    lib.xeng_fengine_create.argtypes = [ctypes.POINTER(FEngineConfig), ctypes.POINTER(vp)]
    lib.xeng_fengine_create.restype = i32
    lib.xeng_fengine_group.argtypes = [vp]
    lib.xeng_fengine_group.restype = i32
    lib.xeng_fengine_run.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    lib.xeng_fengine_run.restype = i32
    lib.xeng_fengine_destroy.argtypes = [vp]
    lib.xeng_fengine_destroy.restype = i32
    lib.xeng_set_fast_autos.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), i32]
    lib.xeng_set_fast_autos.restype = i32
    lib.xeng_dump_fast_autos.argtypes = [vp, pp, i32, i32]
    lib.xeng_dump_fast_autos.restype = i32
    lib.xeng_autotune.argtypes = [vp, pp, i32]
    lib.xeng_autotune.restype = i32
    lib.xeng_graph_create.argtypes = [vp, pp, pp, ctypes.POINTER(vp)]
    lib.xeng_graph_create.restype = i32
    lib.xeng_graph_launch.argtypes = [vp, vp]
    lib.xeng_graph_launch.restype = i32
    lib.xeng_graph_destroy.argtypes = [vp]
    lib.xeng_graph_destroy.restype = i32
    lib.xeng_tuning_save.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    lib.xeng_tuning_save.restype = i32
    lib.xeng_tuning_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    lib.xeng_tuning_load.restype = i32
    lib.xeng_tuning_clear.argtypes = []
    lib.xeng_tuning_clear.restype = i32
    _lib = lib
    return lib


def _check(rc: int):
    if rc != XENG_OK:
        lib = load()
        raise XengError(rc, "%s: %s" % (lib.xeng_strerror(rc).decode(),
                                        lib.xeng_last_error().decode()))


def tri(n: int) -> int:
    return n * (n + 1) // 2


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptrs(values):
    arr = (ctypes.c_void_p * len(values))()
    for k, v in enumerate(values):
        arr[k] = v
    return arr


def tuning_save(path) -> int:
    """xeng_tuning_save: write this process's tuning choices to a JSON file;
    returns the number of entries written."""
    lib = load()
    n = ctypes.c_int32(0)
    _check(lib.xeng_tuning_save(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tuning_load(path) -> int:
    """xeng_tuning_load: merge a tuning file into this process's choices;
    returns the number of entries read."""
    lib = load()
    n = ctypes.c_int32(0)
    _check(lib.xeng_tuning_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tuning_clear():
    """xeng_tuning_clear: forget this process's tuning choices."""
    _check(load().xeng_tuning_clear())


def correlate_dump_static(subarray, samples, out, stream=None):
    """xeng_correlate_dump_static: one subarray's exact sums into out (a
    device int32 tensor [F][tri(N)][2]) without a context and without device
    allocation; enqueued on stream (a torch stream or hipStream_t handle)."""
    lib = load()
    s = subarray if isinstance(subarray, Subarray) else Subarray(
        int(subarray["n_inputs"]), int(subarray["n_chans"]), int(subarray["n_time"]),
        int(subarray.get("in_bits", 4)), int(subarray.get("engine", ENGINE_I8)))
    p = samples if isinstance(samples, int) else samples.data_ptr()
    o = out if isinstance(out, int) else out.data_ptr()
    _check(lib.xeng_correlate_dump_static(ctypes.byref(s), ctypes.c_void_p(p), ctypes.c_void_p(o),
                                          ctypes.c_void_p(_stream_handle(stream))))


class Correlator:
    """X-engine context over one or more subarrays (dicts or Subarray)."""

    def __init__(self, subarrays, stream=None):
        subs = []
        for s in subarrays:
            if isinstance(s, Subarray):
                subs.append(s)
            else:
                subs.append(Subarray(int(s["n_inputs"]), int(s["n_chans"]), int(s["n_time"]),
                                     int(s.get("in_bits", 4)), int(s.get("engine", ENGINE_I8))))
        self.subs = subs
        arr = (Subarray * len(subs))(*subs)
        self._lib = load()
        self._ctx = ctypes.c_void_p()
        _check(self._lib.xeng_create(arr, len(subs), ctypes.c_void_p(_stream_handle(stream)),
                                     ctypes.byref(self._ctx)))

    # -- shapes
    def sample_shape(self, k: int):
        s = self.subs[k]
        base = (s.n_time, s.n_chans, s.n_inputs)
        return base if s.in_bits == 4 else base + (2,)

    def vis_shape(self, k: int):
        s = self.subs[k]
        return (s.n_chans, tri(s.n_inputs), 2)

    # -- calls
    def set_stream(self, stream):
        _check(self._lib.xeng_set_stream(self._ctx, ctypes.c_void_p(_stream_handle(stream))))

    def _sample_ptrs(self, samples):
        if not isinstance(samples, (list, tuple)):
            samples = [samples]
        if len(samples) != len(self.subs):
            raise ValueError("need one sample buffer per subarray")
        ptrs = []
        for k, x in enumerate(samples):
            if isinstance(x, int):
                ptrs.append(x)
                continue
            want = self.sample_shape(k)
            if tuple(x.shape) != want:
                raise ValueError("subarray %d: samples shape %s, expected %s" % (k, tuple(x.shape), want))
            if not x.is_cuda or not x.is_contiguous() or x.element_size() != 1:
                raise ValueError("subarray %d: samples must be a contiguous 1-byte device tensor" % k)
            ptrs.append(x.data_ptr())
        return _ptrs(ptrs)

    def correlate(self, samples):
        """samples: one device tensor (or device pointer int) per subarray."""
        _check(self._lib.xeng_correlate(self._ctx, self._sample_ptrs(samples)))

    def set_kernel(self, kernel: int, k: int = 0, tile: int = 64):
        """Pin subarray k to a kernel family (KERNEL_*); discards accumulated sums."""
        _check(self._lib.xeng_set_kernel(self._ctx, int(k), int(kernel), int(tile)))

    def autotune(self, samples, reps: int = 5):
        """Time the kernel and schedule choices on these samples and keep the fastest."""
        _check(self._lib.xeng_autotune(self._ctx, self._sample_ptrs(samples), int(reps)))

    def capture(self, samples, out):
        """Capture correlate(samples) + dump(out, device, reset) as a replayable Graph."""
        import torch
        if not isinstance(out, (list, tuple)):
            out = [out]
        for k, o in enumerate(out):
            if tuple(o.shape) != self.vis_shape(k) or o.dtype != torch.int32 or not o.is_cuda \
                    or not o.is_contiguous():
                raise ValueError("subarray %d: output must be a contiguous device int32 %s"
                                 % (k, self.vis_shape(k)))
        g = ctypes.c_void_p()
        _check(self._lib.xeng_graph_create(self._ctx, self._sample_ptrs(samples),
                                           _ptrs([o.data_ptr() for o in out]), ctypes.byref(g)))
        return Graph(self._lib, g, self)

    def correlate_dump(self, samples, out=None, reset: bool = True, device: bool = True):
        """correlate(samples) then dump(out, reset, device) in one call (fused
        in the kernel where it can be); returns the list of outputs."""
        out = self._outputs(out, device)
        _check(self._lib.xeng_correlate_dump(self._ctx, self._sample_ptrs(samples),
                                             _ptrs([o.data_ptr() for o in out]),
                                             1 if device else 0, 1 if reset else 0))
        return out

    def _outputs(self, out, device):
        import torch
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device()) if device else torch.device("cpu")
            return [torch.empty(self.vis_shape(k), dtype=torch.int32, device=dev,
                                pin_memory=(not device))
                    for k in range(len(self.subs))]
        if not isinstance(out, (list, tuple)):
            out = [out]
        for k, o in enumerate(out):
            if tuple(o.shape) != self.vis_shape(k) or o.dtype != torch.int32 or not o.is_contiguous():
                raise ValueError("subarray %d: output must be contiguous int32 %s" % (k, self.vis_shape(k)))
            if o.is_cuda != device:
                raise ValueError("subarray %d: output device does not match device=%s" % (k, device))
        return list(out)

    def dump(self, out=None, reset: bool = True, device: bool = True):
        """Copy the sums into out (allocated if None); returns the list of outputs."""
        import torch
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device()) if device else torch.device("cpu")
            out = [torch.empty(self.vis_shape(k), dtype=torch.int32, device=dev,
                               pin_memory=(not device))
                   for k in range(len(self.subs))]
        elif not isinstance(out, (list, tuple)):
            out = [out]
        ptrs = []
        for k, o in enumerate(out):
            if tuple(o.shape) != self.vis_shape(k) or o.dtype != torch.int32 or not o.is_contiguous():
                raise ValueError("subarray %d: output must be contiguous int32 %s" % (k, self.vis_shape(k)))
            if o.is_cuda != device:
                raise ValueError("subarray %d: output device does not match device=%s" % (k, device))
            ptrs.append(o.data_ptr())
        _check(self._lib.xeng_dump(self._ctx, _ptrs(ptrs), 1 if device else 0, 1 if reset else 0))
        return out

    def reset(self):
        _check(self._lib.xeng_dump(self._ctx, None, 1, 1))

    def set_fast_autos(self, inputs, k: int = 0):
        """Select inputs of subarray k whose autocorrelations get a fast cadence."""
        arr = (ctypes.c_int32 * len(inputs))(*[int(i) for i in inputs])
        _check(self._lib.xeng_set_fast_autos(self._ctx, k, arr, len(inputs)))
        self._fast = getattr(self, "_fast", {})
        self._fast[k] = len(inputs)

    def dump_fast_autos(self, reset: bool = True):
        """Re V_ii of the selected inputs, int32 device tensors [n_chans][n] per subarray
        (None for subarrays without a selection)."""
        import torch
        fast = getattr(self, "_fast", {})
        dev = torch.device("cuda", torch.cuda.current_device())
        outs = [torch.empty((s.n_chans, fast[k]), dtype=torch.int32, device=dev)
                if fast.get(k) else None for k, s in enumerate(self.subs)]
        ptrs = _ptrs([o.data_ptr() if o is not None else 0 for o in outs])
        _check(self._lib.xeng_dump_fast_autos(self._ctx, ptrs, 1, 1 if reset else 0))
        return outs

    def samples_since_dump(self, k: int = 0) -> int:
        v = ctypes.c_int64()
        _check(self._lib.xeng_samples_since_dump(self._ctx, k, ctypes.byref(v)))
        return v.value

    def max_dump_samples(self, k: int = 0) -> int:
        v = ctypes.c_int64()
        _check(self._lib.xeng_max_dump_samples(self._ctx, k, ctypes.byref(v)))
        return v.value

    def plan(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(self._lib.xeng_plan_describe(self._ctx, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            rc = self._lib.xeng_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """Streaming integration of one subarray through a device ring of gulps.

    ``host_dumps``: optional list of host int32 tensors ``[F][tri(N)][2]``
    (pinned) that receive dump d in ``host_dumps[d % len]``.
    """

    def __init__(self, subarray, n_slots: int = 4, dump_every: int = 26, host_dumps=None):
        s = subarray if isinstance(subarray, Subarray) else Subarray(
            int(subarray["n_inputs"]), int(subarray["n_chans"]), int(subarray["n_time"]),
            int(subarray.get("in_bits", 4)), int(subarray.get("engine", ENGINE_I8)))
        self.sub = s
        self._lib = load()
        self._host = list(host_dumps) if host_dumps else []
        shape = (s.n_chans, tri(s.n_inputs), 2)
        for h in self._host:
            if tuple(h.shape) != shape or h.is_cuda or not h.is_contiguous():
                raise ValueError("host dump buffers must be contiguous host int32 %s" % (shape,))
        self._s = ctypes.c_void_p()
        hp = _ptrs([h.data_ptr() for h in self._host]) if self._host else None
        _check(self._lib.xeng_stream_create(ctypes.byref(s), n_slots, dump_every, hp,
                                            len(self._host), ctypes.byref(self._s)))

    def next_slot(self):
        """(device pointer of the next gulp's slot, ingest hipStream_t handle);
        (None, None) when a non-blocking stream dropped the gulp."""
        p, st = ctypes.c_void_p(), ctypes.c_void_p()
        rc = self._lib.xeng_stream_next_slot(self._s, ctypes.byref(p), ctypes.byref(st))
        if rc == XENG_EBUSY:
            return None, None
        _check(rc)
        return p.value, st.value

    def drop(self) -> int:
        """Count the next gulp as lost; returns its index."""
        g = ctypes.c_int64()
        _check(self._lib.xeng_stream_drop(self._s, ctypes.byref(g)))
        return g.value

    def set_nonblocking(self, on: bool = True):
        _check(self._lib.xeng_stream_set_nonblocking(self._s, 1 if on else 0))

    def stats(self) -> dict:
        st = StreamStats()
        _check(self._lib.xeng_stream_stats(self._s, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in StreamStats._fields_}

    def set_fast_autos(self, inputs, every: int, host_out=None):
        """Dump the autocorrelations of `inputs` every `every` gulps (host
        int32 tensors [F][len(inputs)], preferably pinned, if given)."""
        arr = (ctypes.c_int32 * len(inputs))(*[int(i) for i in inputs])
        hp = _ptrs([h.data_ptr() for h in host_out]) if host_out else None
        _check(self._lib.xeng_stream_set_fast_autos(self._s, arr, len(inputs), int(every), hp,
                                                   len(host_out) if host_out else 0))
        self._fast_host = list(host_out) if host_out else []

    def fast_wait(self, k: int) -> int:
        """Wait for fast dump k; returns the device pointer of its buffer."""
        p = ctypes.c_void_p()
        _check(self._lib.xeng_stream_fast_wait(self._s, int(k), ctypes.byref(p)))
        return p.value

    def push(self) -> int:
        g = ctypes.c_int64()
        _check(self._lib.xeng_stream_push(self._s, ctypes.byref(g)))
        return g.value

    def dump_wait(self, d: int) -> int:
        """Wait for dump d; returns the device pointer of its dump buffer."""
        p = ctypes.c_void_p()
        _check(self._lib.xeng_stream_dump_wait(self._s, d, ctypes.byref(p)))
        return p.value

    def gulp_times(self, g: int):
        """(arrival -> done ms, filled -> done ms) of gulp g."""
        a, r = ctypes.c_float(), ctypes.c_float()
        _check(self._lib.xeng_stream_gulp_times(self._s, g, ctypes.byref(a), ctypes.byref(r)))
        return a.value, r.value

    def gulps(self) -> int:
        v = ctypes.c_int64()
        _check(self._lib.xeng_stream_gulps(self._s, ctypes.byref(v)))
        return v.value

    def backlog(self) -> int:
        """Gulps pushed whose integration has not finished on the device."""
        v = ctypes.c_int64()
        _check(self._lib.xeng_stream_backlog(self._s, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            rc = self._lib.xeng_stream_destroy(self._s)
            self._s = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured step (correlate + dump + reset) of a Correlator."""

    def __init__(self, lib, handle, owner):
        self._lib, self._g, self._owner = lib, handle, owner

    def launch(self, stream=None):
        _check(self._lib.xeng_graph_launch(self._g, ctypes.c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_g", None) and self._g.value:
            rc = self._lib.xeng_graph_destroy(self._g)
            self._g = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ingest:
    """Corner turn of F-engine packets (format in include/xeng.h) into gulps."""

    def __init__(self, subarray, pkt_time: int, pkt_chans: int, pkt_inputs: int):
        s = subarray if isinstance(subarray, Subarray) else Subarray(
            int(subarray["n_inputs"]), int(subarray["n_chans"]), int(subarray["n_time"]),
            int(subarray.get("in_bits", 4)), int(subarray.get("engine", ENGINE_I8)))
        self.sub = s
        self._lib = load()
        self._ig = ctypes.c_void_p()
        fmt = PacketFormat(pkt_time, pkt_chans, pkt_inputs)
        _check(self._lib.xeng_ingest_create(ctypes.byref(s), ctypes.byref(fmt), ctypes.byref(self._ig)))
        v = ctypes.c_int64()
        _check(self._lib.xeng_ingest_packet_stride(self._ig, ctypes.byref(v)))
        self.stride = v.value

    def gulp(self, packets, n_packets: int, gulp_t0: int, out, stream=None):
        """packets: device uint8 tensor of n_packets * stride bytes; out: device gulp buffer."""
        if packets is not None and packets.numel() < n_packets * self.stride:
            raise ValueError("packet buffer shorter than n_packets * stride")
        shape = (self.sub.n_time, self.sub.n_chans, self.sub.n_inputs)
        if self.sub.in_bits == 8:
            shape = shape + (2,)
        if tuple(out.shape) != shape or not out.is_cuda or not out.is_contiguous() \
                or out.element_size() != 1:
            raise ValueError("out must be a contiguous 1-byte device tensor %s" % (shape,))
        _check(self._lib.xeng_ingest_gulp(self._ig, ctypes.c_void_p(packets.data_ptr() if n_packets else 0),
                                          int(n_packets), int(gulp_t0), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(_stream_handle(stream))))

    def stats(self) -> dict:
        st = IngestStats()
        _check(self._lib.xeng_ingest_stats_get(self._ig, ctypes.byref(st)))
        return dict(received=st.received, missing=st.missing, duplicate=st.duplicate,
                    rejected=st.rejected)

    def close(self):
        if getattr(self, "_ig", None) and self._ig.value:
            rc = self._lib.xeng_ingest_destroy(self._ig)
            self._ig = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FEngine:
    """GPU F-engine (include/xeng.h): 4-tap, 8192-point Hamming PFB, FFT, one
    band gain and 4+4-bit requantisation, written as X-engine input."""

    def __init__(self, n_inputs: int, chan0: int, n_chans: int, gain: float):
        self.cfg = FEngineConfig(int(n_inputs), int(chan0), int(n_chans), float(gain))
        self._lib = load()
        self._fe = ctypes.c_void_p()
        _check(self._lib.xeng_fengine_create(ctypes.byref(self.cfg), ctypes.byref(self._fe)))
        g = self._lib.xeng_fengine_group(self._fe)
        if g < 0:
            _check(g)
        self.group = g

    def run(self, adc, n_spectra: int, out, spec=None, stream=None):
        """adc: device int8 [n_inputs][stride] tensor (rows contiguous); out:
        device uint8 [n_spectra][n_chans][n_inputs]; spec: None or a device
        complex64 tensor of the same shape for the values before rounding."""
        N = self.cfg.n_inputs
        if adc.dim() != 2 or adc.shape[0] != N or adc.element_size() != 1 or not adc.is_cuda \
                or adc.stride(1) != 1:
            raise ValueError("adc must be a device int8 [%d][stride] tensor with unit inner stride" % N)
        shape = (int(n_spectra), self.cfg.n_chans, N)
        for name, tns, es in (("out", out, 1), ("spec", spec, 8)):
            if tns is None:
                continue
            if tuple(tns.shape) != shape or not tns.is_cuda or not tns.is_contiguous() \
                    or tns.element_size() != es:
                raise ValueError("%s must be a contiguous device tensor %s of %d-byte elements"
                                 % (name, shape, es))
        _check(self._lib.xeng_fengine_run(
            self._fe, ctypes.c_void_p(adc.data_ptr()), int(adc.stride(0)), int(n_spectra),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(spec.data_ptr() if spec is not None else 0),
            ctypes.c_void_p(_stream_handle(stream))))

    def run_ptr(self, d_adc: int, adc_stride: int, n_spectra: int, d_out: int, d_spec: int = 0,
                stream=None):
        """run() on raw device pointers (e.g. a streaming ring slot): int8
        [n_inputs][adc_stride] in, uint8 [n_spectra][n_chans][n_inputs] out."""
        _check(self._lib.xeng_fengine_run(self._fe, ctypes.c_void_p(d_adc), int(adc_stride),
                                          int(n_spectra), ctypes.c_void_p(d_out),
                                          ctypes.c_void_p(d_spec or 0),
                                          ctypes.c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_fe", None) and self._fe.value:
            rc = self._lib.xeng_fengine_destroy(self._fe)
            self._fe = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
