"""MI355X-native SH soft-shadow visibility and shading.

Implements the data-parallel path of "Efficient and Differentiable Shadow
Computation for Inverse Problems" (Lyu et al., ICCV 2021) as hand-written HIP
kernels for gfx950 behind a C ABI (include/shvis.h), with a thin Python
binding (``_lib``), a differentiable PyTorch operation (``ops.shade_sh``), a
batched multi-scene solver and a continuous-batching server.
"""
from . import _lib  # noqa: F401  (fails loudly when the HIP library is not built)
from .ops import shade_sh, visibility_sh  # noqa: F401
