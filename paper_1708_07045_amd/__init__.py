"""MI355X-native FFT translational scan for BPMFs and standard binding free
energies (Nguyen, Zhou & Minh).  The compute path is libfftdg.so (HIP,
gfx950); this package is its Python binding."""
from ._lib import (CAP, F32, F64, OCC, PARTIAL_DTYPE, RESULT_DTYPE, EXPORTS, N_FEATURES, N_SCAN_FEATURES, Batch, FFTDG,
                   FFTDGError, GridTools, Network, is_plan, load, LIB_PATH)

__all__ = ["FFTDG", "Batch", "Network", "N_FEATURES", "N_SCAN_FEATURES", "FFTDGError", "load", "PARTIAL_DTYPE", "RESULT_DTYPE", "EXPORTS",
           "LIB_PATH", "is_plan", "GridTools", "F32", "F64", "OCC", "CAP"]
