"""MI355X-native X-engine: exact int8/FP8-MFMA correlation of 4+4-bit voltages,
with the F-engine that produces them (PFB, FFT, 4+4-bit requantisation).

The hot path is the HIP library ``libxeng.so`` (C ABI in ``include/xeng.h``);
this package is its thin Python binding.
"""
from .xeng import (  # noqa: F401
    ENGINE_FP8,
    ENGINE_I8,
    Correlator,
    FEngine,
    Graph,
    Ingest,
    Stream,
    Subarray,
    XengError,
    correlate_dump_static,
    load,
    tri,
    tuning_clear,
    tuning_load,
    tuning_save,
)
