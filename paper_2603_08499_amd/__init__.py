"""MI355X-native VB Gaussian-splatting fit step: E-step + sufficient statistics + conjugate update.

The computation runs in the HIP library ``libvbgs.so`` (C ABI in include/vbgs.h);
this package only marshals arguments to it.
"""
from .vbgs import VBGS, VBGSError, make_params, psnr, query_sizes  # noqa: F401
