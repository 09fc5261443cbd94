"""heatcg: MI355X-native 7-point heat sweep and matrix-free CG.

The compute path is the HIP library ``libheatcg.so`` (kernels for gfx950
behind a C ABI declared in ``include/heatcg.h``); this package only marshals
torch tensors to it.  See ``binding`` for the Python entry points.
"""
from . import inputs  # noqa: F401
from .binding import *  # noqa: F401,F403
