"""MI355X-native SH soft-shadow visibility and shading.

Implements the data-parallel path of "Efficient and Differentiable Shadow
Computation for Inverse Problems" (Lyu et al., ICCV 2021) as hand-written HIP
kernels for gfx950 behind a C ABI (include/shvis.h), with a thin Python
binding (``_lib``), differentiable PyTorch operations (``ops.shade_sh``, and
``ops.shade_sh_channels`` for colour channels sharing one visibility), the
environment-map projection of the lighting (``ops.envmap_to_sh``), a batched
multi-scene solver and a continuous-batching server.
"""
from . import _lib  # noqa: F401  (fails loudly when the HIP library is not built)
from .ops import envmap_to_sh, shade_sh, shade_sh_channels, visibility_sh  # noqa: F401
