"""MI355X-native acoustic full-waveform-inversion hot path (after Cueto et al.,
"Stride", arXiv 2110.03345): forward wave propagation, exact adjoint and vp
gradient as HIP kernels for gfx950 behind a C ABI (include/stride_hip.h).

Layers:
  _abi       ctypes binding of libstride_hip.so (same names as the C ABI) and
             the Plan object
  autograd   StrideWave, a torch.autograd.Function whose backward is the
             adjoint kernel with binomially checkpointed forward wavefields
  serving    continuous-batching solve server
"""
from ._abi import (  # noqa: F401
    LIB_PATH,
    STRIDE_MODE_FORWARD,
    STRIDE_MODE_FORWARD_MEDIUM,
    STRIDE_MODE_GRADIENT,
    STRIDE_MODE_GRADIENT_MEDIUM,
    STRIDE_PATH_BINOMIAL,
    STRIDE_PATH_FULL_HISTORY,
    STRIDE_PATH_SEGMENTED,
    Plan,
    StrideError,
    lib,
    make_grid,
    stride_backward,
    stride_check_finite,
    stride_descent_step,
    stride_forward,
    stride_forward_save,
    stride_gradient,
    stride_gradient_path,
    stride_lowpass,
    stride_plan_create,
    stride_plan_destroy,
    stride_plan_forward,
    stride_plan_forward_medium,
    stride_plan_gradient,
    stride_plan_gradient_medium,
    stride_plan_padded_shape,
    stride_schedule_info,
    stride_timing_enable,
    stride_timing_read,
    stride_workspace_bytes,
    stride_workspace_query,
)
