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
