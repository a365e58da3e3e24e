"""Seeded synthetic inputs for the X-engine: quantised Gaussian voltages.

This package only draws samples and encodes them in the input byte formats
(4+4-bit packed, or 8+8-bit interleaved). It holds none of the correlation
arithmetic, so both the CPU oracle's tests and the GPU path can take their
inputs from it without sharing any of the method.
"""
from .gen import (  # noqa: F401
    BATCH_SHAPES,
    PACKET_MAGIC,
    SEED_BASE,
    TONE_AMP,
    TONE_NU,
    WORKLOADS,
    build,
    drift_phase,
    fixed_tone,
    pack4,
    pack8,
    packet_stride,
    packetize,
    stream,
    thresholds,
    tone_channels,
    tone_series,
    workload,
)
