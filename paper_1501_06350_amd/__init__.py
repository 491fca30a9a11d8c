"""D-Iteration (fluid diffusion) and power iteration for PageRank on MI355X.

The computation lives in the HIP library ``libdi.so`` (C ABI, ``include/di.h``);
``binding`` marshals arguments to it and ``autograd`` wraps the forward solve and
its adjoint as a ``torch.autograd.Function``.
"""
from . import binding  # noqa: F401
from .binding import DIError, Solver, from_graph  # noqa: F401
