"""MI355X-native Laplace-evidence hot path (SunBURST, arXiv 2601.19957).

``synth`` builds seeded synthetic problems; ``_lib`` binds the gfx950 HIP
library (include/sb.h); ``autograd`` exposes the hand-written gradient and
Hessian-vector-product kernels as a differentiable torch function.
"""
from . import synth  # noqa: F401

__all__ = ["synth"]
