"""Pins for the oracle's insertion (scatter) loop and weight application.

Independent references used here: a NumPy brute force over every
(voxel, slice, sample) triple that takes rotations from SciPy, blob values
from SciPy's Bessel function and full-plane values from a NumPy version of
the Hermitian rule (itself pinned against NumPy's complex FFT of real
images); closed forms for axis-aligned slices;
the delta phantom; Hermitian symmetry of the result; the total-weight
identity; linearity and batch/order invariance; and the projection-slice
theorem on an anisotropic Gaussian.
"""
import numpy as np
import pytest
import scipy.special as sp
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import kb

A, ALPHA = 1.9, 15.0


def kb_scipy(d2):
    s = np.clip(1.0 - d2 / (A * A), 0.0, None)
    return np.where(d2 <= A * A, sp.iv(0, ALPHA * np.sqrt(s)) / sp.iv(0, ALPHA), 0.0)


def real_images(rng, S, n):
    return rng.standard_normal((S, n, n))


def hermitian_full(half):
    """Full-plane values [S][ky+h][kx+h] for kx, ky in [-h, h-1] from the half
    plane: stored value for kx > 0 or (kx = 0, ky >= 0), else conj of -k."""
    S, n, w = half.shape
    h = n // 2
    full = np.zeros((S, n, n), dtype=np.complex128)
    ky = np.arange(-h, h)[:, None]
    kx = np.arange(-h, h)[None, :]
    direct = (kx > 0) | ((kx == 0) & (ky >= 0))
    kyd, kxd = np.broadcast_arrays(ky, kx)
    rows = np.where(direct, kyd + h, (-kyd + h) % n)
    cols = np.where(direct, kxd, -kxd)
    ok = cols <= h
    vals = half[:, rows * ok, cols * ok].astype(np.complex128)
    full[:] = np.where(direct, vals, np.conj(vals)) * ok
    return full


def half_and_full(images):
    half = synth.slices_from_projections(images).astype(np.complex64)
    return half, hermitian_full(half)


def test_hermitian_rule_matches_full_fft():
    rng = np.random.default_rng(3)
    n = 16
    imgs = real_images(rng, 3, n)
    half = synth.slices_from_projections(imgs)
    full_fft = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(imgs, axes=(-2, -1))), axes=(-2, -1))
    h = n // 2
    ky, kx = np.meshgrid(np.arange(-h, h), np.arange(-h, h), indexing="ij")
    disk = kx ** 2 + ky ** 2 < h * h
    ext = hermitian_full(half)
    assert np.max(np.abs(ext[:, disk] - full_fft[:, disk])) < 1e-10 * np.max(np.abs(full_fft))


def brute_force(n, full, quats, weight, r_max=None):
    """Every voxel x every slice x every disk sample, straight from the definition."""
    h = n // 2
    r_max = h if r_max is None else r_max
    R = Rotation.from_quat(np.asarray(quats, np.float64)[:, [1, 2, 3, 0]]).as_matrix()
    ks = np.array([(kx, ky) for ky in range(-h, h + 1) for kx in range(-h, h + 1)
                   if kx * kx + ky * ky < r_max * r_max], dtype=np.float64)
    g = np.arange(-h, h + 1)
    vz, vy, vx = np.meshgrid(g, g, g, indexing="ij")
    V = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1).astype(np.float64)
    G = np.zeros(V.shape[0], dtype=np.complex128)
    W = np.zeros(V.shape[0])
    Uv = np.zeros(V.shape[0], dtype=np.int64)
    for s in range(R.shape[0]):
        p = ks[:, 0:1] * R[s][:, 0] + ks[:, 1:2] * R[s][:, 1]          # [Nk,3]
        vals = full[s][ks[:, 1].astype(int) + h, ks[:, 0].astype(int) + h]
        d2 = ((V[:, None, :] - p[None, :, :]) ** 2).sum(-1)
        mask = d2 <= A * A
        w = np.where(mask, weight(d2), 0.0)
        G += w @ vals
        W += w.sum(1)
        Uv += mask.sum(1)
    dim = n + 1
    return G.reshape(dim, dim, dim), W.reshape(dim, dim, dim), Uv.reshape(dim, dim, dim)


@pytest.mark.parametrize("n,S,seed", [(6, 5, 0), (8, 12, 1), (10, 7, 2)])
def test_scatter_matches_brute_force_exact_blob(n, S, seed):
    rng = np.random.default_rng(seed)
    imgs = real_images(rng, S, n)
    half, full = half_and_full(imgs)
    q = synth.random_quaternions(rng, S).astype(np.float32)
    G, W, U = oracle.insert(n, half, q, oracle.Blob(N=0), nthreads=3)
    Gb, Wb, Ub = brute_force(n, full, q.astype(np.float64), kb_scipy)
    assert U == Ub.sum()
    assert oracle.rel_l2(W, Wb) < 1e-13
    assert oracle.rel_l2(G, Gb) < 1e-13


def test_scatter_matches_brute_force_table_rules():
    n, S = 8, 9
    rng = np.random.default_rng(5)
    half, full = half_and_full(real_images(rng, S, n))
    q = synth.random_quaternions(rng, S).astype(np.float32)
    for lerp in (True, False):
        blob = oracle.Blob(N=10000, lerp=lerp)
        T = blob.table()
        G, W, U = oracle.insert(n, half, q, blob)
        Gb, Wb, Ub = brute_force(n, full, q.astype(np.float64),
                                 lambda d2: kb.table_lookup(d2, T, A, lerp=lerp))
        assert U == Ub.sum()
        assert oracle.rel_l2(W, Wb) < 1e-13
        assert oracle.rel_l2(G, Gb) < 1e-13


def test_reduced_cutoff_matches_brute_force():
    n, S = 10, 6
    rng = np.random.default_rng(6)
    half, full = half_and_full(real_images(rng, S, n))
    q = synth.random_quaternions(rng, S).astype(np.float32)
    G, W, U = oracle.insert(n, half, q, oracle.Blob(N=0), r_max=3.3)
    Gb, Wb, Ub = brute_force(n, full, q.astype(np.float64), kb_scipy, r_max=3.3)
    assert U == Ub.sum()
    assert oracle.rel_l2(G, Gb) < 1e-13 and oracle.rel_l2(W, Wb) < 1e-13


def test_per_voxel_form_matches_brute_force():
    n, S = 10, 8
    rng = np.random.default_rng(7)
    half, full = half_and_full(real_images(rng, S, n))
    q = synth.random_quaternions(rng, S).astype(np.float32)
    Gb, Wb, Ub = brute_force(n, full, q.astype(np.float64), kb_scipy)
    vox = rng.integers(-n // 2, n // 2 + 1, size=(200, 3))
    Gv, Wv, Uv = oracle.voxels(n, half, q, vox, oracle.Blob(N=0))
    idx = (vox[:, 2] + n // 2, vox[:, 1] + n // 2, vox[:, 0] + n // 2)
    np.testing.assert_allclose(Wv, Wb[idx], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Gv, Gb[idx], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(Uv.astype(np.int64), Ub[idx])


def test_per_voxel_form_matches_scatter_on_phantom():
    w = synth.make_workload("small", S=40)
    G, W, U = oracle.insert(w.n, w.slices, w.quats)
    rng = np.random.default_rng(8)
    h = w.n // 2
    vox = rng.integers(-h, h + 1, size=(300, 3))
    vox[:20] = rng.integers(-3, 4, size=(20, 3))       # include the dense centre
    Gv, Wv, Uv = oracle.voxels(w.n, w.slices, w.quats, vox)
    idx = (vox[:, 2] + h, vox[:, 1] + h, vox[:, 0] + h)
    np.testing.assert_allclose(Wv, W[idx], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Gv, G[idx], rtol=1e-11, atol=1e-9)


def test_axis_aligned_closed_form():
    # identity orientation: samples sit on lattice points of the plane z = 0
    n, c = 16, 2.5
    h = n // 2
    F = np.full((1, n, h + 1), c, dtype=np.complex64)
    q = np.array([[1.0, 0.0, 0.0, 0.0]], dtype=np.float32)
    b = kb_scipy(np.array([0.0, 1.0, 2.0, 3.0]))
    w0 = b[0] + 4 * b[1] + 4 * b[2]                     # voxel in the plane
    w1 = b[1] + 4 * b[2] + 4 * b[3]                     # voxel one step off the plane
    G, W, U = oracle.insert(n, F, q, oracle.Blob(N=0))
    assert w0 == pytest.approx(1.4936345363, abs=1e-9)
    assert w1 == pytest.approx(0.1496117903, abs=1e-9)
    for x in range(-3, 4):
        for y in range(-3, 4):      # 3x3 neighbourhood inside the disk |k| < 8
            assert W[h, y + h, x + h] == pytest.approx(w0, rel=1e-13)
            assert W[h + 1, y + h, x + h] == pytest.approx(w1, rel=1e-13)
            assert W[h - 1, y + h, x + h] == pytest.approx(w1, rel=1e-13)
    assert np.all(W[: h - 1] == 0) and np.all(W[h + 2:] == 0)
    np.testing.assert_allclose(G, c * W, rtol=1e-14, atol=0)
    # table rule: within the lerp error bound of the exact closed form
    Gt, Wt, _ = oracle.insert(n, F, q, oracle.Blob(N=10000))
    assert Wt[h, h, h] == pytest.approx(w0, abs=1e-6)
    assert Wt[h + 1, h, h] == pytest.approx(w1, abs=1e-6)


def test_delta_phantom_gives_unit_volume():
    # a point at the origin projects to a point; every slice transform is 1
    n, S = 32, 60
    F = np.ones((S, n, n // 2 + 1), dtype=np.complex64)
    q = synth.random_quaternions(np.random.default_rng(9), S).astype(np.float32)
    G, W, U = oracle.insert(n, F, q)
    V = oracle.finalize(G, W)
    mask = W > 0
    assert mask.sum() > 1000
    assert np.max(np.abs(G.imag)) == 0.0
    np.testing.assert_allclose(V[mask], 1.0, rtol=0, atol=1e-13)
    assert np.all(V[~mask] == 0)


def test_hermitian_symmetry_of_result():
    w = synth.make_workload("small", n=32, S=30)
    G, W, U = oracle.insert(w.n, w.slices, w.quats)
    flip = (slice(None, None, -1),) * 3
    assert oracle.rel_l2(np.conj(G[flip]), G) < 1e-13
    assert oracle.rel_l2(W[flip], W) < 1e-13


def test_total_weight_identity():
    w = synth.make_workload("small", n=32, S=25)
    for blob in (oracle.Blob(N=0), oracle.Blob()):
        G, W, U = oracle.insert(w.n, w.slices, w.quats, blob)
        tot = oracle.footprint_total(w.n, w.quats, blob)
        assert W.sum() == pytest.approx(tot, rel=1e-12)
    # sanity: the mean per-pair weight is near the blob's mean over its ball
    assert 0.04 < W.sum() / U < 0.08


def test_linearity_and_weight_independence():
    rng = np.random.default_rng(10)
    n, S = 16, 12
    F1 = synth.slices_from_projections(real_images(rng, S, n)).astype(np.complex64)
    F2 = synth.slices_from_projections(real_images(rng, S, n)).astype(np.complex64)
    c = 0.75
    F12 = (F1.astype(np.complex128) + c * F2.astype(np.complex128)).astype(np.complex64)
    q = synth.random_quaternions(rng, S).astype(np.float32)
    G1, W1, _ = oracle.insert(n, F1, q)
    G2, W2, _ = oracle.insert(n, F2, q)
    G12, W12, _ = oracle.insert(n, F12, q)
    np.testing.assert_array_equal(W1, W2)
    np.testing.assert_array_equal(W1, W12)
    assert oracle.rel_l2(G12, G1 + c * G2) < 1e-6    # complex64 rounding of F12


def test_batching_and_order_invariance():
    w = synth.make_workload("small", n=32, S=40)
    G, W, U = oracle.insert(w.n, w.slices, w.quats)
    Ga, Wa, Ua = oracle.insert(w.n, w.slices[:17], w.quats[:17])
    Gb, Wb, Ub = oracle.insert(w.n, w.slices[17:], w.quats[17:])
    assert Ua + Ub == U
    assert oracle.rel_l2(Ga + Gb, G) < 1e-14 and oracle.rel_l2(Wa + Wb, W) < 1e-14
    perm = np.random.default_rng(11).permutation(w.S)
    Gp, Wp, Up = oracle.insert(w.n, w.slices[perm], w.quats[perm])
    assert Up == U
    assert oracle.rel_l2(Gp, G) < 1e-14 and oracle.rel_l2(Wp, W) < 1e-14


def test_finalize_threshold():
    G = np.array([2 + 2j, 1 + 0j, 5j])
    W = np.array([2.0, 0.0, 1e-3])
    np.testing.assert_array_equal(oracle.finalize(G, W), [1 + 1j, 0, 5000j])
    np.testing.assert_array_equal(oracle.finalize(G, W, tau=1e-2), [1 + 1j, 0, 0])


def test_generator_slice_is_fourier_transform_of_phantom():
    # projection-slice theorem on the generator side: the DFT of the exact
    # projection equals the 3D transform on the plane R (k, 0)^T / n
    n = 64
    rng = np.random.default_rng(12)
    ph = synth.make_phantom(rng, n, 6)
    ph.sigma = np.maximum(ph.sigma, 2.0)
    q = synth.random_quaternions(rng, 4)
    F = synth.slices_from_projections(synth.project(ph, q, n))
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    h = n // 2
    ky, kx = np.meshgrid(np.arange(-h, h), np.arange(0, h + 1), indexing="ij")
    for s in range(4):
        xi = (kx[..., None] * R[s][:, 0] + ky[..., None] * R[s][:, 1]) / n
        ref = synth.phantom_ft(ph, xi)
        assert oracle.rel_l2(F[s], ref) < 1e-4


def _anisotropic_reconstruction(conj_orientation=False):
    n, S = 48, 400
    rng = np.random.default_rng(13)
    ph = synth.Phantom(amp=np.array([1.0]), centers=np.zeros((1, 3)),
                       cov=np.diag([1.5, 2.0, 3.0]) ** 2 * np.ones((1, 3, 3)))
    q = synth.random_quaternions(rng, S)
    F = synth.make_slices(ph, q, n)
    q32 = q.astype(np.float32)
    if conj_orientation:   # a planted convention mistake: R^T instead of R
        q32 = q32 * np.array([1, -1, -1, -1], dtype=np.float32)
    G, W, U = oracle.insert(n, F, q32)
    V = oracle.finalize(G, W)
    h = n // 2
    g = np.arange(-h, h + 1)
    vz, vy, vx = np.meshgrid(g, g, g, indexing="ij")
    xi = np.stack([vx, vy, vz], -1) / n
    ref = synth.phantom_ft(ph, xi)
    mask = (vx ** 2 + vy ** 2 + vz ** 2 <= (n / 4) ** 2) & (W > 0)
    return oracle.rel_l2(V[mask], ref[mask])


def test_projection_slice_theorem_on_anisotropic_gaussian():
    err = _anisotropic_reconstruction()
    assert err < 3e-2          # blob-smoothing limited
    wrong = _anisotropic_reconstruction(conj_orientation=True)
    assert wrong > 10 * err    # the orientation convention is pinned
