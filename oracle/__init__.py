"""FP64 CPU oracle for Kaiser-Bessel Fourier-slice insertion.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only tests/, the package smoke check and the
benchmark's CPU-baseline leg may import or execute it; the product library
never does, and it shares no code with the HIP path.

Contents:
  kb.py        blob profile (power-series I_m), table build and lookup rule
  rotation.py  quaternion -> rotation matrix
  scatter.c    plain FP64 scatter loop, per-voxel sums, footprint totals (C, OpenMP)
  core.py      Python entry points (insert, voxels, finalize, rel_l2, ...)

Every function is pinned by tests against something other than itself
(library routines, brute force on tiny inputs, closed forms, symmetries and
conservation identities).
"""
from .core import Blob, insert, voxels, finalize, rel_l2, blob_values, footprint_total  # noqa: F401
from .kb import bessel_i, kb_profile, kb_table, table_lookup  # noqa: F401
from .rotation import quat_to_matrix  # noqa: F401
