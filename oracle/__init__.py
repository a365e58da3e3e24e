"""CPU oracle for the X-engine (test infrastructure only).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package. The product path never does.
"""
from .oracle import (  # noqa: F401
    accumulate,
    build,
    correlate,
    decode,
    lib_path,
    narrow,
    num_threads,
    projection_check,
    tri,
    unpack_tri,
)
