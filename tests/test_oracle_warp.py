"""Pins of the oracle's displacement operator: identity, integer shifts,
90-degree rotation, a library bilinear resampler, and exact transposition."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import warp
import synth


def test_zero_field_is_identity():
    x = synth.random_image(33, 1).astype(np.float64)
    px, py = warp.field_positions(np.zeros((2, 33, 33)))
    np.testing.assert_array_equal(warp.warp(x, px, py), x)


@pytest.mark.parametrize("ux,uy", [(3, -2), (-5, 4), (0, 7)])
def test_integer_shift_is_roll_with_zero_fill(ux, uy):
    n = 24
    x = synth.random_image(n, 2).astype(np.float64)
    u = np.zeros((2, n, n))
    u[0] = ux
    u[1] = uy
    w = warp.warp(x, *warp.field_positions(u))
    expect = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            rr, cc = r + uy, c + ux
            if 0 <= rr < n and 0 <= cc < n:
                expect[r, c] = x[rr, cc]
    np.testing.assert_array_equal(w, expect)


def test_quarter_turn_is_rot90():
    n = 20
    x = synth.random_image(n, 3).astype(np.float64)
    w = warp.warp(x, *warp.rigid_positions(n, np.pi / 2, 0.0, 0.0))
    np.testing.assert_allclose(w, np.rot90(x), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_matches_library_bilinear(kind):
    n = 64
    x = synth.ellipse_phantom(n, 4).astype(np.float64) + synth.random_image(n, 5).astype(np.float64)
    if kind == "rigid":
        px, py = warp.rigid_positions(n, 0.13, 3.7, -5.2)
    else:
        px, py = warp.field_positions(synth.dilatation_fields(n, 3, 7)[2])
    ref = ndimage.map_coordinates(x, [py, px], order=1, mode="grid-constant", cval=0.0)
    np.testing.assert_allclose(warp.warp(x, px, py), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_adjoint_is_exact_transpose(kind):
    n = 12
    if kind == "rigid":
        px, py = warp.rigid_positions(n, -0.3, 1.25, 0.6)
    else:
        px, py = warp.field_positions(synth.dilatation_fields(n, 2, 9)[1] * 3)
    m = np.zeros((n * n, n * n))
    mt = np.zeros((n * n, n * n))
    e = np.zeros(n * n)
    for q in range(n * n):
        e[:] = 0
        e[q] = 1
        m[:, q] = warp.warp(e.reshape(n, n), px, py).ravel()
        mt[:, q] = warp.warp_adjoint(e.reshape(n, n), px, py).ravel()
    np.testing.assert_allclose(mt, m.T, rtol=0, atol=1e-15)


def test_dot_product_field():
    n = 96
    px, py = warp.field_positions(synth.dilatation_fields(n, 4, 3)[3])
    x = synth.random_image(n, 10).astype(np.float64)
    b = synth.random_image(n, 11).astype(np.float64)
    lhs = float(np.vdot(warp.warp(x, px, py), b))
    rhs = float(np.vdot(x, warp.warp_adjoint(b, px, py)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(b)


def test_position_derivatives_by_differences():
    n, phi, h = 10, 0.21, 1e-6
    d = warp.rigid_position_derivs(n, phi)
    base = np.array(warp.rigid_positions(n, phi, 0.4, -0.3))
    for m in range(3):
        p = [phi, 0.4, -0.3]
        p[m] += h
        num = (np.array(warp.rigid_positions(n, *p)) - base) / h
        np.testing.assert_allclose(num, np.array(d[m]), atol=1e-5)
