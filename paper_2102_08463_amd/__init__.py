"""MI355X-native 1D/2D/3D nonuniform FFTs (types 1, 2 and 3) after cuFINUFFT.

The transforms run in libmnufft.so (hand-written HIP kernels for gfx950 plus
rocFFT for the fine-grid FFT) behind the C ABI in include/mnufft.h; this
package is its thin Python binding.  PyTorch provides device memory and
streams only.
"""
from .plan import Plan, nufft_type1, nufft_type2, nufft_type3  # noqa: F401
from .batch import Batch  # noqa: F401
from . import lib  # noqa: F401

__all__ = ["Plan", "Batch", "nufft_type1", "nufft_type2", "nufft_type3", "lib"]
