"""MI355X-native mixed-precision tile Cholesky of the spherical-harmonic
covariance (arXiv:2408.04440, Sec. III.A.3, III.B, III.D, V.A).

The compute path is libmpchol.so (hand-written HIP for gfx950) behind the C
ABI in include/mpchol.h; `mpchol` is its ctypes binding and `selector` the
training driver of the learned precision selector.
"""
from . import mpchol  # noqa: F401
