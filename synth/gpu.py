"""GPU side of the counter-based generator (synth/gpu_gen.hip).

Draws the same elements as ``synth.stream`` directly into device memory, so a
long stream (the real-time configuration's 10 GB gulps) can be produced on the
device while the host regenerates any channel subset for checking.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .gen import thresholds

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsynth_gpu.so")
SRC = os.path.join(HERE, "gpu_gen.hip")

_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                               "-shared", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops", SRC, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsynth_gpu.so is not built; run synth.gpu.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.synth_fill_device.restype = ctypes.c_int
        lib.synth_fill_device.argtypes = [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        _lib = lib
    return _lib


class DeviceStream:
    """Generator of one stream on the device: ``fill(ptr, t0, n_time, hip_stream)``.

    ``tone`` is ``(amp, phase_fn, tone_chans)`` as for ``synth.stream``. Tone
    threshold tables for times [0, t_total) are built once on the host and
    copied to the device here, so a fill only enqueues the generator kernel
    on the caller's stream (no torch work on streams it does not own).
    """

    def __init__(self, seed: int, n_chans: int, n_inputs: int, in_bits: int, sigma: float,
                 tone=None, t_total: int = 0, device=None):
        import torch
        self.seed, self.F, self.N, self.in_bits, self.sigma = seed, n_chans, n_inputs, in_bits, sigma
        self.lo, self.hi = (-8, 7) if in_bits == 4 else (-127, 127)
        self.n_lv = self.hi - self.lo + 1
        self.dev = device or torch.device("cuda", torch.cuda.current_device())
        self.base = torch.from_numpy(thresholds(self.lo, self.hi, sigma).view(np.int32)).to(self.dev)
        self.tone = tone if tone is not None and tone[2] else None
        self.mask = None
        self.tables = None
        self.t_total = int(t_total)
        if self.tone is not None:
            if self.t_total <= 0:
                raise ValueError("a tone needs t_total, the end of the time range to be drawn")
            m = np.zeros(n_chans, np.uint8)
            m[list(self.tone[2])] = 1
            self.mask = torch.from_numpy(m).to(self.dev)
            amp, phase_fn, _ = self.tone
            chunks = []
            for t0 in range(0, self.t_total, 1 << 20):
                t = np.arange(t0, min(self.t_total, t0 + (1 << 20)), dtype=np.int64)
                ph = phase_fn(t)
                a = np.stack([amp * np.cos(ph), amp * np.sin(ph)], axis=1)
                tab = np.ascontiguousarray(thresholds(self.lo, self.hi, sigma, a)).view(np.int32)
                chunks.append(torch.from_numpy(tab).to(self.dev))
            self.tables = torch.cat(chunks).contiguous()  # [t_total][2][n_lv - 1]
            torch.cuda.synchronize()

    def fill(self, ptr: int, t0: int, n_time: int, hip_stream: int):
        tone_ptr = None
        if self.tables is not None:
            if t0 < 0 or t0 + n_time > self.t_total:
                raise ValueError("times [%d, %d) outside the tone tables [0, %d)" % (
                    t0, t0 + n_time, self.t_total))
            tone_ptr = self.tables.data_ptr() + t0 * 2 * (self.n_lv - 1) * 4
        rc = _load().synth_fill_device(
            ctypes.c_void_p(ptr), self.in_bits, n_time, t0, self.F, self.N,
            ctypes.c_uint64(self.seed & 0xFFFFFFFFFFFFFFFF), self.lo, self.n_lv,
            ctypes.c_void_p(self.base.data_ptr()),
            ctypes.c_void_p(tone_ptr) if tone_ptr else None,
            ctypes.c_void_p(self.mask.data_ptr()) if self.mask is not None else None,
            ctypes.c_void_p(hip_stream))
        if rc != 0:
            raise RuntimeError("synth_fill_device failed: hip error %d" % rc)
