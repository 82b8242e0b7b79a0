"""Pins of the oracle's rigid registration (the preliminary step of
Section I): the gradient against central differences of the energy, recovery
of known rigid motions from exactly warped targets, and the identity."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import registration as reg, warp
import synth


def _ref(n, seed=3, blur=1.5):
    return ndimage.gaussian_filter(synth.ellipse_phantom(n, seed).astype(np.float64), blur)


# (at phi = 0 with an integer shift the samples sit on grid lines, where the
# energy has a kink and the one-sided derivatives differ: not used here)
@pytest.mark.parametrize("theta", [(0.03, 1.2, -0.7), (-0.08, -2.5, 3.1), (0.0, 0.4, 0.3)])
def test_gradient_matches_central_differences(theta):
    n = 48
    ref = _ref(n)
    target = warp.warp(_ref(n, seed=4), *warp.rigid_positions(n, 0.02, 0.5, -0.5))
    E, g = reg.energy_and_grad(ref, target, theta)
    for m, h in enumerate((1e-7, 1e-6, 1e-6)):
        tp, tm = np.array(theta, float), np.array(theta, float)
        tp[m] += h
        tm[m] -= h
        fd = (reg.energy_and_grad(ref, target, tp)[0] - reg.energy_and_grad(ref, target, tm)[0]) / (2 * h)
        assert abs(fd - g[m]) <= 1e-4 * max(abs(g[m]), 1e-3 * np.abs(g).max()), (m, fd, g[m])


@pytest.mark.parametrize("theta", [(0.05, 1.7, -2.3), (-0.087, 3.9, 0.6), (0.02, -4.0, -3.5)])
def test_recovers_known_rigid_motion(theta):
    n = 64
    ref = _ref(n)
    target = warp.warp(ref, *warp.rigid_positions(n, *theta))
    E0, g0 = reg.energy_and_grad(ref, target, theta)
    assert E0 == 0.0 and not g0.any()
    th, E, k = reg.register_rigid(ref, target, max_iter=300, tol=1e-9)
    scale = np.array([(n - 1) / 2.0, 1.0, 1.0])
    assert np.abs((th - np.array(theta)) * scale).max() < 1e-6, (th, theta, k)
    assert E < 1e-12 * np.sum(target ** 2)


def test_identity_target_stays_at_zero():
    ref = _ref(40)
    th, E, k = reg.register_rigid(ref, ref)
    assert not np.asarray(th).any() and E == 0.0 and k == 0


def _rot_affine(phi, tx, ty):
    return (np.cos(phi) - 1.0, -np.sin(phi), np.sin(phi), np.cos(phi) - 1.0, tx, ty)


@pytest.mark.parametrize("theta", [(0.03, 1.2, -0.7), (-0.06, -2.5, 3.1)])
def test_affine_gradient_agrees_with_rigid_chain_rule(theta):
    # a rotation written as an affine map: dE/dphi from the rigid formula equals
    # sum_ab dE/dA_ab dA_ab/dphi from the affine one (two separate derivations)
    n = 48
    ref = _ref(n)
    target = warp.warp(_ref(n, seed=4), *warp.rigid_positions(n, 0.02, 0.5, -0.5))
    E_r, g_r = reg.energy_and_grad(ref, target, theta)
    phi = theta[0]
    E_a, g_a = reg.energy_and_grad_affine(ref, target, _rot_affine(*theta))
    dA = np.array([-np.sin(phi), -np.cos(phi), np.cos(phi), -np.sin(phi)])
    assert abs(E_a - E_r) <= 1e-5 * E_r
    assert abs(g_a[:4] @ dA - g_r[0]) <= 1e-4 * abs(g_r[0])
    np.testing.assert_allclose(g_a[4:], g_r[1:], rtol=1e-4)


def test_affine_gradient_matches_central_differences():
    # steps that move edge samples by 1e-3 px (the field is rounded to float32)
    n = 48
    ref = _ref(n)
    target = warp.warp(_ref(n, seed=4), *warp.field_positions(reg.affine_field(n, (0.01, 0, 0, 0.05, 0, 1))))
    theta = np.array([0.004, -0.01, 0.02, 0.03, 0.6, 0.2])
    E, g = reg.energy_and_grad_affine(ref, target, theta)
    for m in range(6):
        h = 1e-3 / ((n - 1) / 2.0) if m < 4 else 1e-3
        tp, tm = theta.copy(), theta.copy()
        tp[m] += h
        tm[m] -= h
        fd = (reg.energy_and_grad_affine(ref, target, tp)[0] - reg.energy_and_grad_affine(ref, target, tm)[0]) / (2 * h)
        assert abs(fd - g[m]) <= 2e-2 * max(abs(g[m]), 0.1 * np.abs(g[4:]).max()), (m, fd, g[m])


@pytest.mark.parametrize("theta", [(0.0, 0.0, 0.0, 0.06, 0.5, -1.0), _rot_affine(0.05, 1.7, -2.3),
                                   (0.02, 0.0, 0.0, -0.05, -2.0, 0.0)])
def test_affine_recovers_known_maps(theta):
    # linear dilatations (the chest experiment's motion kind) and a rotation
    n = 64
    ref = _ref(n)
    target = warp.warp(ref, *warp.field_positions(reg.affine_field(n, theta)))
    th, E, k = reg.register_affine(ref, target, max_iter=500, tol=1e-9)
    scale = np.array([(n - 1) / 2.0] * 4 + [1.0, 1.0])
    assert np.abs((th - np.array(theta)) * scale).max() < 1e-5, (th, theta, k)


# -- dense displacement fields ------------------------------------------------

def _bump_field(n, ax, ay, sigma):
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    b = np.exp(-((xx - c) ** 2 + (yy - c) ** 2) / (2 * sigma * sigma))
    return np.stack([ax * b, ay * b]).astype(np.float32).astype(np.float64)


def test_field_regulariser_closed_forms():
    # a constant field has no Dirichlet energy; an affine field u_c = a x + b y
    # has a difference a on each of the n (n - 1) horizontal pairs and b on
    # each vertical pair, and L u vanishes away from the border, where it is
    # -a (left column), +a (right column), -b (top row), +b (bottom row)
    n = 9
    R, Lu = reg.field_regulariser(np.full((2, n, n), 1.75))
    assert R == 0.0 and not Lu.any()
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    a, b, a2, b2 = 0.3, -0.2, 0.05, 0.4
    u = np.stack([a * xx + b * yy + 1.0, a2 * xx + b2 * yy - 2.0])
    R, Lu = reg.field_regulariser(u)
    assert np.isclose(R, n * (n - 1) * (a * a + b * b + a2 * a2 + b2 * b2), rtol=1e-13)
    for comp, (ca, cb) in enumerate(((a, b), (a2, b2))):
        L = Lu[comp]
        assert np.allclose(L[1:-1, 1:-1], 0.0, atol=1e-13)
        assert np.allclose(L[1:-1, 0], -ca) and np.allclose(L[1:-1, -1], ca)
        assert np.allclose(L[0, 1:-1], -cb) and np.allclose(L[-1, 1:-1], cb)
        assert np.isclose(L[0, 0], -ca - cb) and np.isclose(L[-1, -1], ca + cb)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_field_gradient_matches_central_differences(lam):
    n = 24
    ref = _ref(n)
    target = warp.warp(_ref(n, seed=4), *warp.field_positions(_bump_field(n, 0.8, -0.6, 5.0)))
    rng = np.random.default_rng(7)
    u = rng.uniform(-0.9, 0.9, size=(2, n, n))
    E, g = reg.energy_and_grad_field(ref, target, u, lam, round32=False)
    h = 1e-6
    for _ in range(12):
        idx = tuple(int(v) for v in (rng.integers(2), rng.integers(n), rng.integers(n)))
        up, um = u.copy(), u.copy()
        up[idx] += h
        um[idx] -= h
        fd = (reg.energy_and_grad_field(ref, target, up, lam, round32=False)[0]
              - reg.energy_and_grad_field(ref, target, um, lam, round32=False)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-5 * np.abs(g).max(), (idx, fd, g[idx])


def test_field_identity_target_stays_at_zero():
    n = 32
    ref = _ref(n)
    u, E, k = reg.register_field(ref, ref.copy(), lam=0.1)
    assert k == 0 and E == 0.0 and not u.any()


def test_field_recovers_smooth_displacement():
    # target = the reference pulled back through a smooth bump displacement
    # (up to 1.2 px); from zero, a weakly regularised descent brings the misfit
    # down by two orders and the field to within ~0.1 px of the truth where
    # the reference has structure (the phantom is piecewise constant, so the
    # displacement along its edges is not determined by the data)
    n = 48
    ref = _ref(n)
    ustar = _bump_field(n, 1.2, -0.8, 10.0)
    target = warp.warp(ref, *warp.field_positions(ustar))
    lam = 0.01
    E0, _ = reg.energy_and_grad_field(ref, target, np.zeros((2, n, n)), lam)
    u, E, k = reg.register_field(ref, target, lam=lam, max_iter=400, tol=1e-4)
    assert E < 2e-2 * E0, (E, E0)
    gm = np.hypot(*np.gradient(ref))
    m = gm > 0.1 * gm.max()
    err = np.sqrt(np.mean(np.sum((u - ustar) ** 2, axis=0)[m]))
    err0 = np.sqrt(np.mean(np.sum(ustar ** 2, axis=0)[m]))
    assert err < 0.15 and err < 0.2 * err0, (err, err0)


@pytest.mark.parametrize("sigma", [0.7, 1.0, 2.5, 4.0])
def test_gaussian_smooth_is_the_library_gaussian_filter(sigma):
    # the scale-space smoothing against scipy's Gaussian filter with the
    # same truncation (radius int(3 sigma + 0.5)) and zero boundary
    rng = np.random.default_rng(1)
    img = rng.standard_normal((37, 37))
    ref = ndimage.gaussian_filter(img, sigma, mode="constant", cval=0.0, truncate=3.0)
    assert np.abs(reg.gaussian_smooth(img, sigma) - ref).max() < 1e-14
    assert np.array_equal(reg.gaussian_smooth(img, 0.0), img)


def test_field_scale_space_schedule():
    # a zero-width schedule is the single level; a coarse-to-fine schedule
    # recovers a displacement of a few pixels that one level leaves far off
    n = 64
    ref = _ref(n, blur=2.0)
    yy = np.mgrid[0:n, 0:n][0].astype(np.float64)
    ustar = _bump_field(n, 1.0, -0.7, 8.0)
    ustar[1] += 1.6 * (yy - (n - 1) / 2.0) / ((n - 1) / 2.0)
    ustar = ustar.astype(np.float32).astype(np.float64)
    target = warp.warp(ref, *warp.field_positions(ustar))
    u1, E1, k1 = reg.register_field(ref, target, lam=0.1, max_iter=120, tol=1e-3)
    u0, E0, k0 = reg.register_field(ref, target, lam=0.1, max_iter=120, tol=1e-3, sigmas=(0.0,))
    assert k0 == k1 and E0 == E1 and np.array_equal(u0, u1)
    us, Es, ks = reg.register_field(ref, target, lam=0.1, max_iter=120, tol=1e-3, sigmas=(4.0, 2.0, 1.0, 0.0))
    gm = np.hypot(*np.gradient(ref))
    m = gm > 0.1 * gm.max()
    rms = lambda v: np.sqrt(np.mean(np.sum(v ** 2, axis=0)[m]))  # noqa: E731
    assert rms(us - ustar) < 0.5 * rms(u1 - ustar), (rms(us - ustar), rms(u1 - ustar))
    assert Es < 0.5 * E1
