"""MI355X-native hot path of self-supervised speed-of-sound and image joint reconstruction for ring-array
photoacoustic computed tomography (Li, Cui, Ma, Alexander, ICCV 2025).

The computation lives in libpact.so (HIP kernels for gfx950 behind the C ABI of include/pact.h); this
package is its ctypes binding (``pact``) and the optimisation driver (``solver``).  The library is loaded
on first use; every call raises PactError if it has not been built (``python -m paper_2409_10876_amd.build``):
there is no fallback implementation.
"""
from . import pact  # noqa: F401
from .pact import PactError, Geometry, load  # noqa: F401

from .solver import (ScanData, PixelGridSolver, NeuralFieldSolver, SirenSolver, BatchedSolver, GroupedBatchSolver,  # noqa: E402,F401,E501
                     SosLoss, geometry_from, prepare_scan)
from . import warmstart  # noqa: E402,F401

__all__ = ["pact", "PactError", "Geometry", "load", "ScanData", "PixelGridSolver", "NeuralFieldSolver", "SirenSolver", "BatchedSolver", "GroupedBatchSolver", "SosLoss",
           "geometry_from", "prepare_scan", "warmstart"]
