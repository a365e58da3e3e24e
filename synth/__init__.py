"""Seeded synthetic inputs: quantised Gaussian voltages for the X-engine and
8-bit ADC samples for the F-engine.

This package only draws samples and encodes them in the input byte formats
(4+4-bit packed, or 8+8-bit interleaved). It holds none of the correlation
arithmetic, so both the CPU oracle's tests and the GPU path can take their
inputs from it without sharing any of the method.
"""
from .gen import (  # noqa: F401
    ADC_FFT,
    ADC_SIGMA,
    ADC_TONES,
    BATCH_SHAPES,
    PACKET_MAGIC,
    SEED_BASE,
    TONE_AMP,
    TONE_NU,
    WORKLOADS,
    adc,
    adc_device,
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
