"""Pins of the oracle's mathematical tools against what the mathematics fixes.

Appendix A (quaternions), Appendix B (B-splines), Appendix C (Algorithms
C1-C3).  Every expected value here comes from an independent textbook route
(vector cross products, Rodrigues' formula, SciPy's B-spline basis, the
closed-form uniform cubic B-splines, LAPACK via NumPy), never from the oracle.
"""
import numpy as np
import pytest

rng = np.random.default_rng(12345)


def _rand_q(n=1):
    q = rng.normal(size=(n, 4))
    return q


def test_quaternion_product_vector_form(oracle_lib):
    # eq:quatmult equals the scalar/vector form eq:quatmultvec
    for a, b in zip(_rand_q(20), _rand_q(20)):
        ab = oracle_lib.qmul(a, b)
        va, vb = a[:3], b[:3]
        vec = np.cross(va, vb) + va * b[3] + vb * a[3]
        sc = a[3] * b[3] - va @ vb
        np.testing.assert_allclose(ab, np.r_[vec, sc], rtol=0, atol=1e-14)


def test_quaternion_identities(oracle_lib):
    for a, b in zip(_rand_q(20), _rand_q(20)):
        ab = oracle_lib.qmul(a, b)
        assert abs(np.linalg.norm(ab) - np.linalg.norm(a) * np.linalg.norm(b)) < 1e-14 * np.linalg.norm(ab)
        np.testing.assert_allclose(oracle_lib.qconj(ab), oracle_lib.qmul(oracle_lib.qconj(b), oracle_lib.qconj(a)),
                                   atol=1e-14)
        np.testing.assert_allclose(oracle_lib.qmul(a, oracle_lib.qinv(a)), [0, 0, 0, 1], atol=1e-15)


def test_vector_rotation_is_rodrigues(oracle_lib):
    for _ in range(20):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(-3, 3)
        q = np.r_[axis * np.sin(ang / 2), np.cos(ang / 2)]
        v = rng.normal(size=3)
        rod = v * np.cos(ang) + np.cross(axis, v) * np.sin(ang) + axis * (axis @ v) * (1 - np.cos(ang))
        np.testing.assert_allclose(oracle_lib.vector_rotate(q, v), rod, atol=1e-14)
        # frame rotation is the inverse (coordinates in the rotated frame)
        np.testing.assert_allclose(oracle_lib.frame_rotate(q, rod), v, atol=1e-14)
        # Q(phi) of eq:qrot is the same quaternion
        np.testing.assert_allclose(oracle_lib.qrot(axis * ang), q if ang > 0 else q, atol=1e-15)


def test_frame_rotation_composition(oracle_lib):
    # eq:quatframerot1: successive frame rotations q1 then q2 equal one by q1 q2
    for _ in range(10):
        q1, q2 = _rand_q(2)
        q1 /= np.linalg.norm(q1)
        q2 /= np.linalg.norm(q2)
        v = rng.normal(size=3)
        two = oracle_lib.frame_rotate(q2, oracle_lib.frame_rotate(q1, v))
        one = oracle_lib.frame_rotate(oracle_lib.qmul(q1, q2), v)
        np.testing.assert_allclose(two, one, atol=1e-14)


def test_quat2mat_orthonormal_and_consistent(oracle_lib):
    for q in _rand_q(20):
        q /= np.linalg.norm(q)
        A = oracle_lib.quat2mat(q)
        np.testing.assert_allclose(A @ A.T, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(A) - 1) < 1e-14
        v = rng.normal(size=3)
        # attitude matrix maps celestial to instrument coordinates (eq:attmat)
        np.testing.assert_allclose(A @ v, oracle_lib.frame_rotate(q, v), atol=1e-14)
    # rotation about Z by theta: SRS x axis = (cos, sin, 0) in celestial coordinates
    th = 0.3
    A = oracle_lib.quat2mat([0, 0, np.sin(th / 2), np.cos(th / 2)])
    np.testing.assert_allclose(A[0], [np.cos(th), np.sin(th), 0], atol=1e-15)


def _scipy_basis(knots, t):
    """Values at t of all cubic B-splines on the knots, from SciPy's
    B-spline design matrix (an independent library implementation)."""
    from scipy.interpolate import BSpline
    return BSpline.design_matrix(np.atleast_1d(t), knots, 3).toarray()[0]


def _knots(K=12, dt=7.0, t0=-40.0):
    inner = t0 + dt * np.arange(K + 1)
    return np.r_[np.full(3, t0), inner, np.full(3, inner[-1])]


def test_left_index(oracle_lib):
    k = _knots()
    N = k.size - 4
    assert oracle_lib.left_index(k, k[3]) == 3
    assert oracle_lib.left_index(k, k[5] + 1e-9) == 5
    assert oracle_lib.left_index(k, k[6]) == 6            # tau_l <= t
    assert oracle_lib.left_index(k, k[6] - 1e-12) == 5
    assert oracle_lib.left_index(k, k[N]) == N - 1        # end of the spline interval


def test_bspline_basis(oracle_lib):
    """The four non-zero cubic B-splines equal SciPy's basis on a regular
    sequence with 4-fold end knots and on an irregular one (a double knot
    included); partition of unity; non-negative."""
    rng_k = np.random.default_rng(3)
    inner = np.cumsum(rng_k.uniform(0.5, 9.0, 14)) - 40.0
    inner[6] = inner[5]                                   # a double knot
    irregular = np.r_[np.full(3, inner[0]), inner, np.full(3, inner[-1])]
    for k in (_knots(), irregular):
        N = k.size - 4
        for t in np.linspace(k[3], k[N] - 1e-9, 97):
            ell = oracle_lib.left_index(k, t)
            b = oracle_lib.bspline(k, ell, t)
            assert np.all(b >= 0)
            assert abs(b.sum() - 1) < 1e-15                    # partition of unity
            ref = _scipy_basis(k, t)
            np.testing.assert_allclose(b, ref[ell - 3:ell + 1], atol=4e-16)
            assert np.abs(np.delete(ref, np.arange(ell - 3, ell + 1))).max(initial=0.0) == 0.0
    k = _knots()
    # uniform interior interval: textbook cubic B-spline pieces
    for u in np.linspace(0, 1, 11)[:-1]:
        ell = 7
        t = k[ell] + u * 7.0
        b = oracle_lib.bspline(k, ell, t)
        ref = [(1 - u) ** 3 / 6, (3 * u**3 - 6 * u**2 + 4) / 6, (-3 * u**3 + 3 * u**2 + 3 * u + 1) / 6, u**3 / 6]
        np.testing.assert_allclose(b, ref, atol=1e-15)


def test_bspline_c2_continuity(oracle_lib):
    k = _knots()
    # value, first and second derivative continuous at a simple knot
    h = 1e-4
    for kn in [6, 7, 9]:
        def spl(t):
            ell = oracle_lib.left_index(k, t)
            c = np.zeros(k.size - 4)
            c[ell - 3:ell + 1] = oracle_lib.bspline(k, ell, t)
            return c
        left = [spl(k[kn] - j * h) for j in (1, 2, 3)]
        right = [spl(k[kn] + j * h) for j in (0, 1, 2)]
        val_l = 3 * left[0] - 3 * left[1] + left[2]      # quadratic extrapolation to the knot
        np.testing.assert_allclose(val_l, right[0], atol=1e-10)


def _psd(n, r):
    X = rng.normal(size=(n, r))
    return X @ X.T


def test_cholesky_spd_matches_lapack(oracle_lib):
    for n in (1, 2, 5, 16, 40):
        A = _psd(n, n + 3) + n * np.eye(n)
        b = rng.normal(size=n)
        U, x, d = oracle_lib.chol_solve(A, b)
        assert d == 0
        L = np.linalg.cholesky(A)
        np.testing.assert_allclose(np.triu(U), L.T, rtol=1e-13, atol=1e-13 * np.abs(L).max())
        np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)


def test_cholesky_semidefinite_rho(oracle_lib):
    """Rank-deficient PSD matrices: the modified algorithm gives a valid
    solution (rho_b of Appendix C.3 of order 1e4 at the 99th percentile)."""
    u = 2.0**-52
    rho = []
    for _ in range(200):
        n = int(rng.integers(4, 30))
        r = int(rng.integers(1, n))
        N = _psd(n, r)
        xt = rng.normal(size=n)
        b = N @ xt
        U, x, d = oracle_lib.chol_solve(N, b)
        assert np.all(np.isfinite(x))
        rho.append(np.linalg.norm(b - N @ x) / (u * np.linalg.norm(b)))
    assert np.percentile(rho, 99) < 1e7
    assert np.median(rho) < 1e4


def test_cholesky_zero_rows_defect(oracle_lib):
    A = _psd(6, 8) + np.eye(6)
    A[2, :] = 0
    A[:, 2] = 0
    b = rng.normal(size=6)
    b[2] = 0
    U, x, d = oracle_lib.chol_solve(A, b)
    assert d == 1 and x[2] == 0
    keep = [0, 1, 3, 4, 5]
    np.testing.assert_allclose(x[keep], np.linalg.solve(A[np.ix_(keep, keep)], b[keep]), rtol=1e-11)


def test_band_equals_dense_bitwise(oracle_lib):
    n, hb = 60, 15
    X = rng.normal(size=(n + 40, n))
    # band matrix: zero outside |i - j| <= hb
    A = X.T @ X
    mask = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= hb
    A = np.where(mask, A, 0.0) + 5 * n * np.eye(n)
    b = rng.normal(size=n)
    UB = np.zeros((n, hb + 1))
    for j in range(n):
        for k in range(hb + 1):
            if j + k < n:
                UB[j, k] = A[j, j + k]
    Ud, xd, dd = oracle_lib.chol_solve(A, b)
    Ub, xb, db = oracle_lib.band_solve(UB, b, hb)
    assert dd == db == 0
    assert np.array_equal(xd, xb)
    for j in range(n):
        for k in range(hb + 1):
            if j + k < n:
                assert Ub[j, k] == Ud[j, j + k]
