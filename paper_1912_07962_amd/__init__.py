"""slimLS (sampled limited-memory row-action least squares) for MI355X.

The hot path -- matrix-free Joseph projectors, Gram blocks, FP64 Cholesky /
PCG of the Gram system and the fused update -- lives in the HIP library
``_lib/libslim.so`` behind the C ABI of ``include/slim.h``; ``slim`` is its
ctypes binding.
"""
from .slim import (  # noqa: F401
    Cnn, Group, Slim, Slim3D, SlimError, cnn_layout, header_symbols, load,
)
