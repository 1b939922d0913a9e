"""MI355X-native Parallel Toplesets Propagation (geodesic distances on
triangle meshes, arXiv 1810.08218).

The computation lives in the HIP library ``libptp.so`` behind the C ABI of
``include/ptp.h``; ``ptp`` is its ctypes binding and ``inputs`` builds the
seeded synthetic meshes.
"""
from .ptp import (BAND_FIXED_HALF, BAND_JACOBI, BAND_PAPER, PTP_EDEVICE, PTP_EINVAL, PTP_ENOCONV,
                  PTP_ENOMEM, PTP_EUNSUPPORTED, PTP_OK, Batch, MeshDesc, Plan, PTPError, Schedule,
                  Solution, concat, load, solve)

__all__ = ["Plan", "Batch", "MeshDesc", "Schedule", "concat", "PTPError", "Solution", "load",
           "solve", "PTP_OK", "PTP_EINVAL", "PTP_ENOMEM", "PTP_EDEVICE", "PTP_ENOCONV",
           "PTP_EUNSUPPORTED", "BAND_PAPER", "BAND_FIXED_HALF", "BAND_JACOBI"]
