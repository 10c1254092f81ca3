"""MI355X-native model-based iterative edge-illumination (EI) tomography.

The compute path is a C-ABI shared library (libeitomo.so, declared in
include/eitomo.h) of hand-written HIP kernels for gfx950. The Python binding
(`ops`) is argument marshalling over it: torch supplies device memory and streams,
every step of the reconstruction runs in the library's kernels. The library is
loaded on first use and a missing build raises instead of falling back.
"""
from .configs import SliceConfig, BatchConfig, SMALL_64, SLICE_512, SLICE_1024, BATCH_256  # noqa: F401
