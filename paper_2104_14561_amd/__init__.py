"""MI355X-native backward Feynman-Kac scheme for exit-time probabilities.

The compute path is libfkexit.so (hand-written HIP for gfx950, C ABI in
include/fkexit.h); ``fkexit`` marshals arguments and uses PyTorch only for
device memory and streams.
"""
from .fkexit import (FkError, Plan, gh_rule, load, precision_probe, probe_lds_atomics,  # noqa: F401
                     solve, tune)
