"""Pins for the oracle's blob profile, table rule and rotations.

Each check compares against something other than the oracle itself: SciPy's
Bessel and rotation routines, closed-form special values, or the exactness of
linear interpolation on a linear table.
"""
import numpy as np
import pytest
import scipy.special as sp
from scipy.spatial.transform import Rotation

import oracle
from oracle import kb
from oracle.rotation import quat_to_matrix

A, ALPHA = 1.9, 15.0


def kb_scipy(d2, a=A, alpha=ALPHA, m=0):
    d2 = np.asarray(d2, dtype=np.float64)
    s = np.clip(1.0 - d2 / (a * a), 0.0, None)
    v = s ** (0.5 * m) * sp.iv(m, alpha * np.sqrt(s)) / sp.iv(m, alpha)
    return np.where(d2 <= a * a, v, 0.0)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_bessel_series_matches_scipy(m):
    x = np.linspace(0.0, 40.0, 201)
    ref = sp.iv(m, x)
    got = kb.bessel_i(m, x)
    mask = ref > 0
    assert np.max(np.abs(got[mask] / ref[mask] - 1.0)) < 1e-13
    assert np.all(got[~mask] == 0.0)


def test_bessel_i0_matches_numpy_i0():
    x = np.linspace(0.0, 20.0, 77)
    assert np.max(np.abs(kb.bessel_i(0, x) / np.i0(x) - 1)) < 1e-13


@pytest.mark.parametrize("m", [0, 2])
@pytest.mark.parametrize("alpha", [10.0, 15.0])
def test_profile_python_and_c_match_scipy(m, alpha):
    d2 = np.linspace(0.0, A * A * 1.05, 1001)
    ref = kb_scipy(d2, A, alpha, m)
    py = kb.kb_profile(d2, A, alpha, m)
    c = oracle.blob_values(d2, oracle.Blob(a=A, alpha=alpha, m=m, N=0))
    big = ref > 1e-300
    assert np.max(np.abs(py[big] / ref[big] - 1)) < 1e-13
    assert np.max(np.abs(c[big] / ref[big] - 1)) < 1e-13
    assert np.all(py[d2 > A * A] == 0) and np.all(c[d2 > A * A] == 0)


def test_profile_special_values():
    # b(0) = 1 (normalisation), b(a^2) = 1 / I0(alpha) for order 0, b = 0 beyond a
    vals = kb.kb_profile([0.0, A * A, A * A * (1 + 1e-12), 100.0], A, ALPHA, 0)
    assert vals[0] == pytest.approx(1.0, abs=1e-15)
    assert vals[1] == pytest.approx(1.0 / np.i0(ALPHA), rel=1e-13)
    assert vals[2] == 0.0 and vals[3] == 0.0
    d2 = np.linspace(0, A * A, 5000)
    assert np.all(np.diff(kb.kb_profile(d2, A, ALPHA)) < 0)


def test_table_endpoints_and_lerp_error_bound():
    N = 10000
    T = kb.kb_table(A, ALPHA, 0, N)
    assert T[0] == pytest.approx(1.0, abs=1e-15)
    assert T[-1] == pytest.approx(1.0 / np.i0(ALPHA), rel=1e-13)
    rng = np.random.default_rng(0)
    d2 = rng.uniform(0.0, A * A, 1_000_000)
    exact = kb_scipy(d2)
    lerp = kb.table_lookup(d2, T, A, lerp=True)
    trunc = kb.table_lookup(d2, T, A, lerp=False)
    assert np.max(np.abs(lerp - exact)) < 1e-7
    # truncation is far coarser; the rule matters at the 1e-5 level
    assert np.max(np.abs(trunc - exact)) > 1e-4


def test_table_lerp_is_exact_on_linear_table():
    # linear interpolation reproduces a linear function: pins index and fraction
    N = 37
    T = 3.0 - 2.0 * np.arange(N) / (N - 1)          # value = 3 - 2 d^2 / a^2
    d2 = np.linspace(0.0, A * A, 999)
    got = kb.table_lookup(d2, T, A, lerp=True)
    np.testing.assert_allclose(got, 3.0 - 2.0 * d2 / (A * A), rtol=0, atol=1e-14)
    # truncation returns the node at or below t
    t = d2 * (N - 1) / (A * A)
    np.testing.assert_allclose(kb.table_lookup(d2, T, A, lerp=False),
                               3.0 - 2.0 * np.floor(t) / (N - 1), atol=1e-14)


def test_c_table_lookup_matches_python_rule():
    rng = np.random.default_rng(1)
    d2 = np.concatenate([rng.uniform(0, A * A * 1.1, 20000), [0.0, A * A]])
    for lerp in (True, False):
        blob = oracle.Blob(N=10000, lerp=lerp)
        c = oracle.blob_values(d2, blob)
        py = kb.table_lookup(d2, blob.table(), A, lerp=lerp)
        np.testing.assert_allclose(c, py, rtol=0, atol=1e-15)


def test_rotation_matches_scipy_and_is_proper():
    rng = np.random.default_rng(2)
    q = rng.standard_normal((500, 4))
    R = quat_to_matrix(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # SciPy is scalar-last
    np.testing.assert_allclose(R, ref, atol=1e-14)
    eye = np.einsum("sji,sjk->sik", R, R)
    np.testing.assert_allclose(eye, np.broadcast_to(np.eye(3), eye.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    np.testing.assert_allclose(quat_to_matrix(-q), R, atol=1e-15)
    np.testing.assert_allclose(quat_to_matrix(3.7 * q), R, atol=1e-14)


def test_rotation_about_z_turns_x_axis():
    for th in (0.3, 1.0, 2.5):
        R = quat_to_matrix([np.cos(th / 2), 0.0, 0.0, np.sin(th / 2)])
        np.testing.assert_allclose(R @ [1.0, 0.0, 0.0], [np.cos(th), np.sin(th), 0.0], atol=1e-15)


@pytest.mark.parametrize("bad", [[0, 0, 0, 0], [np.nan, 0, 0, 1], [np.inf, 1, 0, 0]])
def test_rotation_rejects_degenerate(bad):
    with pytest.raises(ValueError):
        quat_to_matrix(bad)
