"""MI355X-native out-of-core stencil sweep (SO2DR method: region sharing in
HBM plus redundant halo computation so that kernels can fuse time steps).

The work happens in libso2dr.so (hand-written gfx950 HIP kernels, C++
planner and stream executor) behind the C interface in include/so2dr.h;
this package only marshals arguments.  Importing it does not load the
library; the first plan does, and fails loudly if it is missing."""
from .plan import (Plan, stencil_offsets, adjoint_buffers_needed, suggest,  # noqa: F401
                   pinned_empty)
from ._lib import So2drError  # noqa: F401


def __getattr__(name):
    if name == "StencilLoss":   # imports torch lazily
        from .autograd import StencilLoss
        return StencilLoss
    raise AttributeError(name)
