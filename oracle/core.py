"""Python entry points of the FP64 CPU oracle (test infrastructure only).

Wraps the plain C scatter loop in scatter.c (built into liboracle.so by
oracle/build.py) and adds the weight-application step.  Follows the paper's
Algorithm 1 "3D reconstruction" (Sect. 5.3.1): zero G and W, insert the
slices, apply the weights W to G.  Every function takes the same inputs the
product library takes (complex64 half-plane slices and FP32 quaternions) and
returns FP64 results over the full centered (n+1)^3 box.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from .kb import kb_table
from .rotation import quat_to_matrix

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

BLOB_EXACT, BLOB_TABLE_LERP, BLOB_TABLE_TRUNC = 0, 1, 2


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint64)
        ci, cd = ctypes.c_int, ctypes.c_double
        lib.oracle_insert.argtypes = [ci, ci, fp, dp, cd, cd, ci, ci, dp, ci, cd, dp, dp, up, up, ci]
        lib.oracle_insert.restype = ci
        lib.oracle_voxels.argtypes = [ci, ci, fp, dp, cd, cd, ci, ci, dp, ci, cd, ci, ip, dp, dp, up, ci]
        lib.oracle_voxels.restype = ci
        lib.oracle_blob.argtypes = [ci, dp, cd, cd, ci, ci, dp, ci, dp]
        lib.oracle_blob.restype = ci
        lib.oracle_footprint_total.argtypes = [ci, ci, dp, cd, cd, ci, ci, dp, ci, cd, dp]
        lib.oracle_footprint_total.restype = ci
        _lib = lib
    return _lib


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass(frozen=True)
class Blob:
    """Blob parameters: radius a, taper alpha, order m, table size N
    (N = 0 selects the exact profile) and lookup rule."""
    a: float = 1.9
    alpha: float = 15.0
    m: int = 0
    N: int = 10000
    lerp: bool = True

    @property
    def mode(self) -> int:
        if self.N == 0:
            return BLOB_EXACT
        return BLOB_TABLE_LERP if self.lerp else BLOB_TABLE_TRUNC

    def table(self) -> np.ndarray:
        if self.N == 0:
            return np.zeros(2, dtype=np.float64)
        return np.ascontiguousarray(kb_table(self.a, self.alpha, self.m, self.N))


def _prep(n, slices, quats):
    n = int(n)
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    slices = np.ascontiguousarray(slices, dtype=np.complex64)
    S = slices.shape[0] if slices.ndim == 3 else 0
    if S and slices.shape[1:] != (n, n // 2 + 1):
        raise ValueError(f"slices must be [S][{n}][{n // 2 + 1}]")
    quats = np.asarray(quats, dtype=np.float32).reshape(-1, 4)
    if quats.shape[0] != S:
        raise ValueError("one quaternion per slice")
    R = np.ascontiguousarray(quat_to_matrix(quats.astype(np.float64)).reshape(S, 9)) if S else np.zeros((0, 9))
    return n, S, slices, R


def insert(n, slices, quats, blob: Blob = Blob(), r_max=None, nthreads=None, with_half=False):
    """Scatter all slices into the full box.  Returns (G complex128 [(n+1)]^3,
    W float64 [(n+1)]^3, U = number of (sample, voxel) pairs within the blob);
    with_half=True appends the number of those pairs whose voxel has x >= 0."""
    lib = _load()
    n, S, slices, R = _prep(n, slices, quats)
    r_max = 0.5 * n if r_max is None else float(r_max)
    dim = n + 1
    G = np.zeros((dim, dim, dim, 2), dtype=np.float64)
    W = np.zeros((dim, dim, dim), dtype=np.float64)
    U = ctypes.c_uint64(0)
    Uh = ctypes.c_uint64(0)
    table = blob.table()
    nthreads = nthreads or min(8, os.cpu_count() or 1)
    fl = slices.view(np.float32)
    rc = lib.oracle_insert(n, S, _ptr(fl, ctypes.c_float), _ptr(R, ctypes.c_double),
                           blob.a, blob.alpha, blob.m, blob.mode, _ptr(table, ctypes.c_double),
                           int(blob.N), r_max, _ptr(G, ctypes.c_double), _ptr(W, ctypes.c_double),
                           ctypes.byref(U), ctypes.byref(Uh), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_insert failed ({rc})")
    out = (G[..., 0] + 1j * G[..., 1], W, int(U.value))
    return out + (int(Uh.value),) if with_half else out


def voxels(n, slices, quats, vox, blob: Blob = Blob(), r_max=None, nthreads=None):
    """Per-voxel sums for voxels vox [nv][3] = centered (x, y, z).
    Returns (G [nv] complex128, W [nv] float64, U [nv] uint64)."""
    lib = _load()
    n, S, slices, R = _prep(n, slices, quats)
    r_max = 0.5 * n if r_max is None else float(r_max)
    vox = np.ascontiguousarray(vox, dtype=np.int32).reshape(-1, 3)
    nv = vox.shape[0]
    Gv = np.zeros((nv, 2), dtype=np.float64)
    Wv = np.zeros(nv, dtype=np.float64)
    Uv = np.zeros(nv, dtype=np.uint64)
    table = blob.table()
    nthreads = nthreads or min(8, os.cpu_count() or 1)
    fl = slices.view(np.float32)
    rc = lib.oracle_voxels(n, S, _ptr(fl, ctypes.c_float), _ptr(R, ctypes.c_double),
                           blob.a, blob.alpha, blob.m, blob.mode, _ptr(table, ctypes.c_double),
                           int(blob.N), r_max, nv, _ptr(vox, ctypes.c_int),
                           _ptr(Gv, ctypes.c_double), _ptr(Wv, ctypes.c_double),
                           _ptr(Uv, ctypes.c_uint64), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_voxels failed ({rc})")
    return Gv[:, 0] + 1j * Gv[:, 1], Wv, Uv


def blob_values(d2, blob: Blob = Blob()):
    """Blob weights from the C implementation (exact series or table rule)."""
    lib = _load()
    d2 = np.ascontiguousarray(d2, dtype=np.float64).ravel()
    out = np.zeros_like(d2)
    table = blob.table()
    rc = lib.oracle_blob(d2.size, _ptr(d2, ctypes.c_double), blob.a, blob.alpha, blob.m,
                         blob.mode, _ptr(table, ctypes.c_double), int(blob.N),
                         _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_blob failed")
    return out


def footprint_total(n, quats, blob: Blob = Blob(), r_max=None):
    """sum over slices and disk samples of the blob weight deposited in the box."""
    lib = _load()
    quats = np.asarray(quats, dtype=np.float32).reshape(-1, 4)
    S = quats.shape[0]
    R = np.ascontiguousarray(quat_to_matrix(quats.astype(np.float64)).reshape(S, 9)) if S else np.zeros((0, 9))
    r_max = 0.5 * n if r_max is None else float(r_max)
    table = blob.table()
    out = ctypes.c_double(0.0)
    rc = lib.oracle_footprint_total(int(n), S, _ptr(R, ctypes.c_double), blob.a, blob.alpha,
                                    blob.m, blob.mode, _ptr(table, ctypes.c_double), int(blob.N),
                                    r_max, ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_footprint_total failed")
    return out.value


def finalize(G, W, tau: float = 0.0):
    """Apply the weights: V = G / W where W > tau, else 0 (FP64)."""
    G = np.asarray(G, dtype=np.complex128)
    W = np.asarray(W, dtype=np.float64)
    V = np.zeros_like(G)
    mask = W > tau
    V[mask] = G[mask] / W[mask]
    return V


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 over all elements (FP64)."""
    x = np.asarray(x).astype(np.complex128).ravel()
    ref = np.asarray(ref).astype(np.complex128).ravel()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    return float(num / den) if den > 0 else float(num)
