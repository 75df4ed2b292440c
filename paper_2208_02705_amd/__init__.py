"""MI355X (gfx950) hot path of 360Roam's geometry-aware radiance fields.

Equirect/pinhole ray generation -> occupied-voxel sampling -> routing by
field -> positional encoding + per-field MLP (MFMA) -> alpha compositing,
plus the backward pass for fine-tuning, the global field, Stage I
occupancy estimation, Stage II field assignment and the distillation of
the global field into the local ones; every step is a HIP kernel in
libr360.so behind the C ABI of include/r360.h. This package only marshals
arguments (ctypes) and provides torch.autograd wrappers. The shared library
is loaded on first use and its absence is an error.
"""
from ._lib import R360Error, FP32, BF16, FP16, FP64_GRADCHECK, LIB_PATH  # noqa: F401
from .render import (Scene, Equirect, EquirectRenderer, PinholeRenderer, RenderFunction, GradcheckFunction,  # noqa: F401
                     sample_rays, render_rays, render_equirect, render_pinhole, render_stereo, backward, train_step, adam_step,
                     pinhole_rays,
                     field_params, field_frames, lr_at, profile_enable, profile_read, GlobalField)
from .occupancy import OccupancyMap, depth_uncertainty, global_measure  # noqa: F401
from .assign import assign_fields, assign_uniform  # noqa: F401
from .distill import global_points, distill_step  # noqa: F401
