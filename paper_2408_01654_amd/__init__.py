"""MI355X-native Gauss-Newton bundle adjustment over DPV-SLAM's patch graph.

The numeric work runs in the HIP library libdpvba.so (C ABI in
include/dpvba.h); ``binding`` marshals torch device tensors into it.
"""
from .binding import (  # noqa: F401
    FP32, FP64, MIXED, BatchTensors, Context, DpvbaError, GraphTensors, LIB_PATH, bundle_adjust, bundle_adjust_many,
    lib, solve_backward_many, solve_many, status_string,
)
