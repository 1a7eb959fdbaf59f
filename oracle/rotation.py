"""Orientation of a Fourier slice, FP64 (oracle; test infrastructure only).

The paper inserts 2D samples "of arbitrary orientation" (Sect. 4.2, "3D Fourier
Reconstruction") without fixing a representation.  Orientations here are unit
quaternions q = (w, x, y, z), scalar first, normalised before use; R(q) is the
active Hamilton rotation matrix, and slice sample k = (kx, ky) sits at the
volume frequency R (kx, ky, 0)^T.  q and -q describe the same rotation.
"""
from __future__ import annotations

import numpy as np


def quat_to_matrix(q) -> np.ndarray:
    """R(q) for q of shape [..., 4] (w, x, y, z); returns [..., 3, 3] in FP64."""
    q = np.asarray(q, dtype=np.float64)
    norm = np.sqrt(np.sum(q * q, axis=-1, keepdims=True))
    if np.any(~np.isfinite(norm)) or np.any(norm == 0.0):
        raise ValueError("quaternion must be finite and non-zero")
    q = q / norm
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3), dtype=np.float64)
    R[..., 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[..., 0, 1] = 2.0 * (x * y - w * z)
    R[..., 0, 2] = 2.0 * (x * z + w * y)
    R[..., 1, 0] = 2.0 * (x * y + w * z)
    R[..., 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[..., 1, 2] = 2.0 * (y * z - w * x)
    R[..., 2, 0] = 2.0 * (x * z - w * y)
    R[..., 2, 1] = 2.0 * (y * z + w * x)
    R[..., 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R
