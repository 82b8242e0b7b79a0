"""Pins of the oracle's ray transform against facts that do not depend on it:
axis-aligned special cases, the closed-form sinogram of a disc, a brute-force
hat-function formulation, and exact transposition."""
import math

import numpy as np
import pytest

from oracle import projector
import synth


@pytest.mark.parametrize("n,na,nd", [(16, 12, 24), (32, 40, 46), (128, 120, 182)])
def test_theta0_is_column_sums(n, na, nd):
    x = synth.random_image(n, 5).astype(np.float64)
    s = projector.forward(x, na, nd)
    off = (nd - n) // 2
    expect = np.zeros(nd)
    expect[off:off + n] = x.sum(axis=0)
    np.testing.assert_allclose(s[0], expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,na,nd", [(16, 12, 24), (32, 40, 46), (128, 120, 182)])
def test_theta90_is_row_sums(n, na, nd):
    x = synth.random_image(n, 6).astype(np.float64)
    s = projector.forward(x, na, nd)
    off = (nd - n) // 2
    expect = np.zeros(nd)
    expect[off:off + n] = x.sum(axis=1)
    np.testing.assert_allclose(s[na // 2], expect, rtol=0, atol=1e-10)


def _disc_error(n, na, nd, a, b, R):
    img = synth.disc_image(n, a, b, R, supersample=8)
    s = projector.forward(img, na, nd)
    th = np.pi * np.arange(na) / na
    t = np.arange(nd) - (nd - 1) / 2
    arg = R ** 2 - (t[None, :] - a * np.cos(th)[:, None] - b * np.sin(th)[:, None]) ** 2
    exact = 2 * np.sqrt(np.maximum(arg, 0))
    return np.linalg.norm(s - exact) / np.linalg.norm(exact), s, exact


def test_off_centre_disc_matches_closed_form():
    # A uniform disc of radius R centred at (a, b) has line integral
    # 2 sqrt(R^2 - (t - a cos - b sin)^2) on the ray at distance t, angle theta.
    # The discretisation error of a pixelated disc is first order in the pixel
    # size: halving the pixel (same disc in physical units) halves it.
    e64, _, _ = _disc_error(64, 60, 92, 8.65, -10.8, 11.5)
    e128, s, exact = _disc_error(128, 60, 182, 17.3, -21.6, 23.0)
    assert e128 < 1.5e-2, e128
    assert 1.6 < e64 / e128 < 2.6, (e64, e128)
    # a mirrored disc (a -> -a) gives a visibly different sinogram: the sign of the geometry
    img2 = synth.disc_image(128, -17.3, -21.6, 23.0, supersample=8)
    s2 = projector.forward(img2, 60, 182)
    assert np.linalg.norm(s2 - exact) / np.linalg.norm(exact) > 0.3


def _brute_force(x, na, nd):
    """Pure-Python loops: every pixel of every line along the stepping axis
    contributes the hat function of its distance to the ray's crossing."""
    n = x.shape[0]
    half = (n - 1) / 2
    out = np.zeros((na, nd))
    for k in range(na):
        th = math.pi * k / na
        cs, sn = math.cos(th), math.sin(th)
        rows = abs(cs) >= abs(sn) - 1e-15
        for j in range(nd):
            t = j - (nd - 1) / 2
            acc = 0.0
            for line in range(n):
                u = line - half
                cross = (t - u * sn) / cs + half if rows else (t - u * cs) / sn + half
                for pix in range(n):
                    w = max(0.0, 1.0 - abs(cross - pix))
                    acc += w * (x[line, pix] if rows else x[pix, line])
            out[k, j] = acc / (abs(cs) if rows else abs(sn))
    return out


def test_brute_force_hat_formulation():
    x = synth.random_image(7, 9).astype(np.float64)
    na, nd = 9, 11     # angles avoid the 45-degree tie, where the two rules differ
    s = projector.forward(x, na, nd)
    np.testing.assert_allclose(s, _brute_force(x, na, nd), rtol=0, atol=1e-12)


def test_adjoint_is_exact_transpose_16():
    n, na, nd = 16, 12, 24
    m = projector.matrix(n, na, nd)
    mt = np.zeros((n * n, na * nd))
    e = np.zeros(na * nd)
    for q in range(na * nd):
        e[:] = 0
        e[q] = 1
        mt[:, q] = projector.adjoint(e.reshape(na, nd), n).ravel()
    np.testing.assert_allclose(mt, m.T, rtol=0, atol=1e-14)
    # every column of the matrix touches at most 2 pixels per angle per line
    assert (np.count_nonzero(m, axis=1) <= 2 * n).all()


@pytest.mark.parametrize("n,na,nd", [(64, 80, 92), (128, 120, 182)])
def test_dot_product(n, na, nd):
    x = synth.random_image(n, 1).astype(np.float64)
    y = synth.random_sinograms(1, na, nd, 2)[0].astype(np.float64)
    lhs = float(np.vdot(projector.forward(x, na, nd), y))
    rhs = float(np.vdot(x, projector.adjoint(y, n)))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(projector.forward(x, na, nd)) * np.linalg.norm(y)


def test_single_ray_and_pixel_helpers():
    n, na, nd = 48, 36, 70
    x = synth.random_image(n, 3).astype(np.float64)
    y = synth.random_sinograms(1, na, nd, 4)[0].astype(np.float64)
    s = projector.forward(x, na, nd)
    b = projector.adjoint(y, n)
    for (k, j) in [(0, 10), (9, 35), (18, 40), (27, 60), (35, 1)]:
        assert abs(projector.ray_sum(x, na, nd, k, j) - s[k, j]) < 1e-11
    for (r, c) in [(0, 0), (10, 30), (47, 47), (24, 5)]:
        assert abs(projector.backproject_pixel(y, n, r, c) - b[r, c]) < 1e-10


def test_stepping_axis_integer_rule():
    th, rows = projector.angle_table(720)
    assert rows[180] and rows[540] and not rows[181] and not rows[539]
    assert rows.sum() == 361   # k = 0..180 and 540..719


@pytest.mark.parametrize("n,na,nd", [(16, 12, 23), (17, 13, 25)])
def test_sparse_matrix_equals_dense_matrix(n, na, nd):
    # the sparse assembly holds exactly the weights of `forward`, column by column
    m = projector.sparse_matrix(n, na, nd)
    assert m.shape == (na * nd, n * n)
    np.testing.assert_array_equal(m.toarray(), projector.matrix(n, na, nd))


@pytest.mark.parametrize("n,na,nd", [(64, 60, 92), (63, 45, 70), (48, 72, 40)])
def test_sparse_matrix_products_are_forward_and_adjoint(n, na, nd):
    # its product is the transform and its transpose's product is the scatter
    # of the same weights (including a detector narrower than the image)
    m = projector.sparse_matrix(n, na, nd)
    x = synth.random_image(n, 31).astype(np.float64)
    y = synth.random_sinograms(1, na, nd, 32)[0].astype(np.float64)
    a = (m @ x.ravel()).reshape(na, nd)
    b = (m.T @ y.ravel()).reshape(n, n)
    np.testing.assert_allclose(a, projector.forward(x, na, nd), rtol=0, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(b, projector.adjoint(y, n), rtol=0, atol=1e-12 * np.abs(b).max())


def test_matrix_backed_operators_equal_plain_ones():
    from oracle.operators import GatedOperators
    n, na, nd = 40, 36, 58
    params = synth.rigid_params(2, 3, 8.0, 3.0)
    plain = GatedOperators(n, na, nd, "rigid", params)
    fast = GatedOperators(n, na, nd, "rigid", params, matrix=projector.sparse_matrix(n, na, nd))
    x = synth.random_image(n, 4).astype(np.float64)
    y = synth.random_sinograms(1, na, nd, 5)[0].astype(np.float64)
    for i in range(2):
        np.testing.assert_allclose(fast.A(i, x), plain.A(i, x), rtol=0, atol=1e-12 * np.abs(plain.A(i, x)).max())
        np.testing.assert_allclose(fast.At(i, y), plain.At(i, y), rtol=0, atol=1e-12 * np.abs(plain.At(i, y)).max())
    with pytest.raises(ValueError):
        GatedOperators(n, na, nd, "rigid", params, matrix=projector.sparse_matrix(n, na, nd + 1))
