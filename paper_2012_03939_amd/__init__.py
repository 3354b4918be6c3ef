"""MI355X-native differentiable path tracer (Shape from Tracing, Sec. 3.2-3.3).

The compute path is the HIP library ``libshapetrace.so`` (C ABI in
``include/shapetrace.h``); :mod:`.binding` marshals torch tensors into it and
:mod:`.autograd` exposes it as a ``torch.autograd.Function``.
"""
from . import scenes  # noqa: F401  (seeded synthetic inputs)

__all__ = ["scenes", "binding", "autograd"]
