"""Seeded phantoms, orientations and Fourier slices (FP64 generation).

Phantom: K Gaussians f(x) = sum_j A_j exp(-(x-c_j)^T S_j^-1 (x-c_j) / 2) in a
box of n pixels per side, pixel (h, h, h) at the origin (h = n/2).  The
projection in orientation q is the exact line integral

    P_q(u) = integral f(R(q) (u_x, u_y, t)^T) dt,

sampled at u = (col - h, row - h), where R(q) is the active rotation of the
unit quaternion q = (w, x, y, z).  The slice is the centered 2D DFT of P_q in
Hermitian half-plane layout [row = ky + h][kx], kx in [0, h]:
rfft2(ifftshift(P)) then fftshift along rows, rounded to complex64.

Rotations are applied here with quaternion products (q* v q rotates by R^T),
not with a matrix, so this module shares no arithmetic with either side of the
insertion.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import os

import numpy as np
import scipy.fft

_FFT_WORKERS = max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# quaternions
# --------------------------------------------------------------------------
def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def _conj(q: np.ndarray) -> np.ndarray:
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def _inverse_rotation_matrices(quats: np.ndarray) -> np.ndarray:
    """M_s = R(q_s)^T built column by column as q* e_i q.  [S,3,3]."""
    q = np.asarray(quats, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    S = q.shape[0]
    M = np.empty((S, 3, 3))
    for i in range(3):
        e = np.zeros((S, 4))
        e[:, 1 + i] = 1.0
        M[:, :, i] = _qmul(_qmul(_conj(q), e), q)[:, 1:]
    return M


def random_quaternions(rng: np.random.Generator, S: int) -> np.ndarray:
    """Haar-uniform rotations: normalised 4D standard normal vectors (FP64)."""
    q = rng.standard_normal((S, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def clustered_quaternions(rng: np.random.Generator, S: int, q0, sigma_deg: float = 3.0) -> np.ndarray:
    """Views near q0: q = q0 (x) (cos(t/2), sin(t/2) axis), axis uniform on the
    sphere, t = |N(0, sigma)|."""
    q0 = np.asarray(q0, dtype=np.float64)
    q0 = q0 / np.linalg.norm(q0)
    axis = rng.standard_normal((S, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    t = np.abs(rng.standard_normal(S)) * np.deg2rad(sigma_deg)
    dq = np.concatenate([np.cos(t / 2)[:, None], np.sin(t / 2)[:, None] * axis], axis=1)
    return _qmul(np.broadcast_to(q0, dq.shape), dq)


# --------------------------------------------------------------------------
# phantom
# --------------------------------------------------------------------------
@dataclass
class Phantom:
    amp: np.ndarray                 # [K]
    centers: np.ndarray             # [K,3] (x, y, z) in pixels from the box centre
    sigma: np.ndarray | None = None  # [K] isotropic widths, or None
    cov: np.ndarray | None = None    # [K,3,3] general covariances, or None

    def covariances(self) -> np.ndarray:
        if self.cov is not None:
            return self.cov
        return (self.sigma ** 2)[:, None, None] * np.eye(3)[None]


def make_phantom(rng: np.random.Generator, n: int, K: int) -> Phantom:
    """K isotropic Gaussians: A ~ U[0.5, 1], sigma ~ U[1.5, max(1.5, n/16)],
    centres uniform in the ball of radius n/4."""
    amp = rng.uniform(0.5, 1.0, K)
    sigma = rng.uniform(1.5, max(1.5, n / 16.0), K)
    d = rng.standard_normal((K, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = (n / 4.0) * rng.uniform(0.0, 1.0, K) ** (1.0 / 3.0)
    return Phantom(amp=amp, centers=d * r[:, None], sigma=sigma)


def phantom_ft(ph: Phantom, xi: np.ndarray) -> np.ndarray:
    """Continuous 3D Fourier transform f^(xi) = integral f(x) exp(-2 pi i xi.x) dx
    at frequencies xi [..., 3] (cycles per pixel)."""
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros(xi.shape[:-1], dtype=np.complex128)
    covs = ph.covariances()
    for A, c, C in zip(ph.amp, ph.centers, covs):
        det = np.linalg.det(C)
        quad = np.einsum("...i,ij,...j->...", xi, C, xi)
        out += A * (2 * np.pi) ** 1.5 * np.sqrt(det) * np.exp(-2 * np.pi ** 2 * quad) \
            * np.exp(-2j * np.pi * (xi @ c))
    return out


def project(ph: Phantom, quats: np.ndarray, n: int) -> np.ndarray:
    """Exact line-integral projections [S][n][n] (FP64, row = u_y + h, col = u_x + h)."""
    h = n // 2
    M = _inverse_rotation_matrices(quats)             # R^T
    S = M.shape[0]
    u = np.arange(n, dtype=np.float64) - h
    cprime = np.einsum("sij,kj->ski", M, ph.centers)   # [S,K,3] = R^T c
    if ph.cov is None:
        amp = ph.amp * np.sqrt(2 * np.pi) * ph.sigma          # [K]
        inv2s2 = 1.0 / (2.0 * ph.sigma ** 2)                  # [K]
        gx = np.exp(-(u[None, None, :] - cprime[:, :, 0:1]) ** 2 * inv2s2[None, :, None])
        gy = np.exp(-(u[None, None, :] - cprime[:, :, 1:2]) ** 2 * inv2s2[None, :, None])
        gy *= amp[None, :, None]
        return np.matmul(gy.transpose(0, 2, 1), gx)           # [S, row, col]
    # general covariance: marginal of the rotated Gaussian over the t axis
    out = np.zeros((S, n, n))
    uy, ux = np.meshgrid(u, u, indexing="ij")
    for A, C, cp in zip(ph.amp, ph.cov, np.transpose(cprime, (1, 0, 2))):
        Cr = np.einsum("sia,ab,sjb->sij", M, C, M)          # R^T C R
        Cuu = Cr[:, :2, :2]
        det3 = np.linalg.det(C)
        det2 = np.linalg.det(Cuu)
        inv = np.linalg.inv(Cuu)
        dx = ux[None] - cp[:, 0, None, None]
        dy = uy[None] - cp[:, 1, None, None]
        q = inv[:, 0, 0, None, None] * dx * dx + 2 * inv[:, 0, 1, None, None] * dx * dy \
            + inv[:, 1, 1, None, None] * dy * dy
        out += (A * (2 * np.pi) ** 1.5 * np.sqrt(det3) / (2 * np.pi * np.sqrt(det2)))[:, None, None] \
            * np.exp(-0.5 * q)
    return out


def slices_from_projections(P: np.ndarray) -> np.ndarray:
    """Centered DFT of each projection in half-plane layout [S][n][n/2+1] (complex128).

    SciPy's FFT is the same pocketfft code as NumPy's, run on several threads."""
    F = scipy.fft.rfft2(np.fft.ifftshift(P, axes=(-2, -1)), axes=(-2, -1), workers=_FFT_WORKERS)
    return np.fft.fftshift(F, axes=-2)


def make_slices(ph: Phantom, quats: np.ndarray, n: int, chunk: int = 1000) -> np.ndarray:
    """complex64 [S][n][n/2+1] slices of the phantom for the given orientations."""
    S = quats.shape[0]
    out = np.empty((S, n, n // 2 + 1), dtype=np.complex64)
    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)
        out[s0:s1] = slices_from_projections(project(ph, quats[s0:s1], n))
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    n: int
    slices: np.ndarray          # complex64 [S][n][n/2+1]
    quats: np.ndarray           # float32 [S][4]
    phantom: Phantom
    meta: dict = field(default_factory=dict)

    @property
    def S(self) -> int:
        return int(self.quats.shape[0])


# name -> (n, S, K, phantom seed, orientation seed, clustered fraction)
WORKLOADS = {
    "small": (64, 500, 20, 1, 2, 0.0),
    "paper": (128, 10000, 40, 3, 4, 0.0),
    "precision": (256, 50000, 40, 7, 8, 0.1),
}


def make_workload(name: str = "small", n: int | None = None, S: int | None = None,
                  K: int | None = None, seed_phantom: int | None = None,
                  seed_orient: int | None = None, clustered: float | None = None) -> Workload:
    """Build a named workload, optionally overriding its sizes or seeds.

    Orientations are Haar-uniform; a fraction `clustered` of them (the last
    ones) lie within a few degrees of one random view.  Quaternions are
    rounded to FP32 before projecting so that the projections match exactly
    the orientations handed to the insertion step."""
    base = WORKLOADS.get(name, WORKLOADS["small"])
    n = base[0] if n is None else int(n)
    S = base[1] if S is None else int(S)
    K = base[2] if K is None else int(K)
    sp = base[3] if seed_phantom is None else int(seed_phantom)
    so = base[4] if seed_orient is None else int(seed_orient)
    cl = base[5] if clustered is None else float(clustered)
    ph = make_phantom(np.random.default_rng(sp), n, K)
    rng = np.random.default_rng(so)
    n_cl = int(round(cl * S))
    q = random_quaternions(rng, S - n_cl)
    if n_cl:
        q0 = random_quaternions(rng, 1)[0]
        q = np.concatenate([q, clustered_quaternions(rng, n_cl, q0)], axis=0)
    quats = q.astype(np.float32)
    slices = make_slices(ph, quats.astype(np.float64), n)
    return Workload(name=name, n=n, slices=slices, quats=quats, phantom=ph,
                    meta=dict(K=K, seed_phantom=sp, seed_orient=so, clustered=cl))


# name -> (boxes, slice-count range, seed of the counts, K): several
# reconstructions of uneven sizes inserted together; job j uses phantom seed
# 50 + j and orientation seed 60 + j
BATCHES = {
    "batch8": ((64, 96, 128, 160, 192, 224, 256, 256), (2000, 20000), 5, 40),
}


def batch_specs(name: str = "batch8") -> list:
    """(n, S, K, seed_phantom, seed_orient) of each job of a named batch; the
    slice counts are drawn uniformly from the range with the batch's seed."""
    boxes, (lo, hi), seed, K = BATCHES[name]
    counts = np.random.default_rng(seed).integers(lo, hi + 1, size=len(boxes))
    return [(int(n), int(S), K, 50 + j, 60 + j) for j, (n, S) in enumerate(zip(boxes, counts))]


def batch_quaternions(spec) -> np.ndarray:
    """The FP32 orientations make_workload draws for one job of a batch
    (without building its slices)."""
    n, S, K, sp, so = spec
    return random_quaternions(np.random.default_rng(so), S).astype(np.float32)


# --------------------------------------------------------------------------
# 16-bit slice storage (the storage formats the library accepts)
# --------------------------------------------------------------------------
def _f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 to bfloat16 (round to nearest, ties to even); returns uint16 bits."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    rounded = b + np.uint32(0x7FFF) + lsb
    return (rounded >> 16).astype(np.uint16)


def quantize_slices(slices: np.ndarray, fmt: str):
    """Store complex64 slices as 16-bit (re, im) pairs.

    fmt = "f16": IEEE half values of F / scale_s with one FP32 scale per slice,
    chosen as max(|re|, |im|) / 32768 (so the largest component maps to 32768,
    well inside the half range); fmt = "bf16": bfloat16 values, scale 1.
    Returns (bits uint16 [S][n][n/2+1][2], scales float32 [S])."""
    sl = np.ascontiguousarray(slices, dtype=np.complex64)
    S = sl.shape[0]
    comp = sl.view(np.float32).reshape(sl.shape + (2,))
    if fmt == "f16":
        peak = np.abs(comp).reshape(S, -1).max(axis=1)
        scales = np.where(peak > 0, peak / 32768.0, 1.0).astype(np.float32)
        q = (comp / scales[:, None, None, None]).astype(np.float16)
        return q.view(np.uint16), scales
    if fmt == "bf16":
        return _f32_to_bf16_bits(comp), np.ones(S, dtype=np.float32)
    raise ValueError("fmt must be 'f16' or 'bf16'")


def dequantize_slices(bits: np.ndarray, scales: np.ndarray, fmt: str) -> np.ndarray:
    """Exact complex64 values of 16-bit stored slices (what the kernels read)."""
    if fmt == "f16":
        comp = bits.view(np.float16).astype(np.float32) * scales[:, None, None, None].astype(np.float32)
    elif fmt == "bf16":
        comp = (bits.astype(np.uint32) << 16).view(np.float32)
    else:
        raise ValueError("fmt must be 'f16' or 'bf16'")
    comp = np.ascontiguousarray(comp, dtype=np.float32)
    return comp.view(np.complex64).reshape(bits.shape[:-1])
