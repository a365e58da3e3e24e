"""ctypes wrapper around the plain-C oracle ``xcorr_oracle.c``.

TEST INFRASTRUCTURE ONLY: the product path must never import this module.

The C file is the definition of the visibility sums (Section 2, Fig. 2
caption; Section 2.5), decoded from the 4+4-bit format of Section 2.2 or the
8+8-bit form of Section 2.4, summed exactly in int64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain -O2 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        lib.oracle_decode.argtypes = [vp, i32, i64, vp, vp]
        lib.oracle_decode.restype = i32
        lib.oracle_accumulate.argtypes = [vp, i32, i64, i32, i32, vp, i32, vp]
        lib.oracle_accumulate.restype = i32
        lib.oracle_narrow.argtypes = [vp, vp, i64]
        lib.oracle_narrow.restype = i64
        lib.oracle_projection_check.argtypes = [vp, i32, i64, i32, i32, i32, vp, vp]
        lib.oracle_projection_check.restype = i64
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        _lib = lib
    return _lib


def tri(n: int) -> int:
    return n * (n + 1) // 2


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _check_stream(samples: np.ndarray, in_bits: int):
    if in_bits == 4:
        if samples.dtype != np.uint8 or samples.ndim != 3:
            raise ValueError("4-bit stream must be uint8 [T][F][N]")
        T, F, N = samples.shape
    elif in_bits == 8:
        if samples.dtype != np.int8 or samples.ndim != 4 or samples.shape[3] != 2:
            raise ValueError("8-bit stream must be int8 [T][F][N][2]")
        T, F, N, _ = samples.shape
    else:
        raise ValueError("in_bits must be 4 or 8")
    if not samples.flags.c_contiguous:
        raise ValueError("stream must be C-contiguous")
    return T, F, N


def decode(samples: np.ndarray, in_bits: int):
    """Integer (re, im) of every sample, int32, shape of the stream without the pair axis."""
    samples = np.ascontiguousarray(samples)
    shape = samples.shape if in_bits == 4 else samples.shape[:-1]
    n = int(np.prod(shape))
    re = np.empty(n, np.int32)
    im = np.empty(n, np.int32)
    rc = _load().oracle_decode(samples.ctypes.data, in_bits, n, re.ctypes.data, im.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_decode failed")
    return re.reshape(shape), im.reshape(shape)


def accumulate(acc: np.ndarray, samples: np.ndarray, in_bits: int, chans=None) -> np.ndarray:
    """acc (int64 [n_sel][tri(N)][2]) += sums over this stream, in place."""
    T, F, N = _check_stream(samples, in_bits)
    if chans is None:
        n_sel, cptr = F, None
        carr = None
    else:
        carr = np.ascontiguousarray(np.asarray(chans, np.int32))
        n_sel, cptr = len(carr), carr.ctypes.data
    if acc.dtype != np.int64 or acc.shape != (n_sel, tri(N), 2) or not acc.flags.c_contiguous:
        raise ValueError("acc must be C-contiguous int64 [%d][%d][2]" % (n_sel, tri(N)))
    rc = _load().oracle_accumulate(samples.ctypes.data, in_bits, T, F, N, cptr, n_sel,
                                   acc.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_accumulate failed (%d)" % rc)
    return acc


def correlate(samples: np.ndarray, in_bits: int, chans=None) -> np.ndarray:
    """int64 [n_sel][tri(N)][2] visibility sums of one stream."""
    T, F, N = _check_stream(samples, in_bits)
    n_sel = F if chans is None else len(chans)
    acc = np.zeros((n_sel, tri(N), 2), np.int64)
    return accumulate(acc, samples, in_bits, chans)


def narrow(acc: np.ndarray) -> np.ndarray:
    """int64 sums -> int32 output words; raises if any value does not fit."""
    acc = np.ascontiguousarray(acc, np.int64)
    out = np.empty(acc.shape, np.int32)
    over = _load().oracle_narrow(acc.ctypes.data, out.ctypes.data, acc.size)
    if over:
        raise OverflowError("%d visibility words exceed int32" % over)
    return out


def projection_check(samples: np.ndarray, in_bits: int, chan: int, vis_chan: np.ndarray,
                     w: np.ndarray) -> int:
    """Rows of V w that disagree with sum_t x (x^H w) for one channel (0 = consistent)."""
    T, F, N = _check_stream(samples, in_bits)
    vis_chan = np.ascontiguousarray(vis_chan, np.int32)
    if vis_chan.shape != (tri(N), 2):
        raise ValueError("vis_chan must be int32 [tri(N)][2]")
    w = np.ascontiguousarray(w, np.int64)
    if w.shape != (N, 2):
        raise ValueError("w must be int64 [N][2]")
    r = _load().oracle_projection_check(samples.ctypes.data, in_bits, T, F, N, chan,
                                        vis_chan.ctypes.data, w.ctypes.data)
    if r < 0:
        raise ValueError("oracle_projection_check: bad arguments")
    return int(r)


def unpack_tri(vis: np.ndarray, n: int) -> np.ndarray:
    """Packed lower triangle [..., tri(N), 2] -> full Hermitian complex128 [..., N, N]."""
    vis = np.asarray(vis)
    lead = vis.shape[:-2]
    out = np.zeros(lead + (n, n), np.complex128)
    ii, jj = np.tril_indices(n)
    k = ii * (ii + 1) // 2 + jj
    v = vis[..., k, 0].astype(np.float64) + 1j * vis[..., k, 1].astype(np.float64)
    out[..., ii, jj] = v
    out[..., jj, ii] = np.conj(v)
    return out
