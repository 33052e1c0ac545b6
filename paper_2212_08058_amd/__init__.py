"""MI355X-native space-time power iteration (spectral video segmentation hot path).

The compute path is the HIP library libstpi.so (C ABI in include/stpi.h);
this package only marshals torch tensors (device memory) and streams into it.
"""
from .api import (Kernel, launch_shape, power_iterate, problem_for, step, step_noalloc, time_chain_step, time_step,  # noqa: F401
                  workspace_bytes)
from ._native import StpiError  # noqa: F401
