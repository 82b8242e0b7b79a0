"""Pins of the oracle gradient through unrolled SPDHG: central finite
differences of the loss itself (FP64), for the starting image and for rigid and
field motion parameters, and the Jacobian transpose identity."""
import numpy as np
import pytest

from oracle import grad, spdhg
from oracle.operators import GatedOperators
import synth


def _setup(kind, n=12, na=14, nd=18, N=3):
    if kind == "rigid":
        params = synth.rigid_params(N, 4, 6.0, 1.5)
    else:
        # a constant sub-pixel offset keeps every sample off the grid lines,
        # where the bilinear interpolant has kinks
        params = synth.dilatation_fields(n, N, 5).astype(np.float64) * 0.3 + np.array([0.37, -0.21])[None, :, None, None]
    ops = GatedOperators(n, na, nd, kind, params)
    x_true = synth.ellipse_phantom(n, 2).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((N, na, nd), 3))
    alpha = 2.0
    sig, tau, th, _ = spdhg.step_sizes_spdhg([500.0] * N, alpha, N)
    p = [1.0 / N] * N
    seq = [0, 2, 1, 2, 0]
    x0 = 0.5 * x_true + 0.1 * synth.random_image(n, 7).astype(np.float64)
    return ops, params, d, alpha, sig, tau, th, p, seq, x0, x_true


@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_grad_wrt_start_image_by_differences(kind):
    ops, params, d, alpha, sig, tau, th, p, seq, x0, xt = _setup(kind)
    L, gx, _ = grad.unrolled_loss_and_grad(ops, x0, d, alpha, sig, tau, th, p, seq, xt)
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.standard_normal(x0.shape)
        h = 1e-3
        lp = grad.unrolled_loss(ops, x0 + h * v, d, alpha, sig, tau, th, p, seq, xt)
        lm = grad.unrolled_loss(ops, x0 - h * v, d, alpha, sig, tau, th, p, seq, xt)
        fd = (lp - lm) / (2 * h)        # exact for a quadratic up to rounding
        assert abs(fd - float(np.vdot(gx, v))) < 1e-8 * max(1.0, abs(fd))


def test_grad_wrt_rigid_params_by_differences():
    ops, params, d, alpha, sig, tau, th, p, seq, x0, xt = _setup("rigid")
    L, _, gm = grad.unrolled_loss_and_grad(ops, x0, d, alpha, sig, tau, th, p, seq, xt)
    # the loss is piecewise smooth in the motion (bilinear kinks at grid lines);
    # a small step stays within one piece for almost every pixel
    for h, tol in [(1e-6, 1e-4)]:
        for i in range(3):
            for m in range(3):
                pp, pm = params.copy(), params.copy()
                pp[i, m] += h
                pm[i, m] -= h
                lp = grad.unrolled_loss(GatedOperators(12, 14, 18, "rigid", pp), x0, d, alpha, sig, tau, th, p, seq, xt)
                lm = grad.unrolled_loss(GatedOperators(12, 14, 18, "rigid", pm), x0, d, alpha, sig, tau, th, p, seq, xt)
                fd = (lp - lm) / (2 * h)
                scale = np.abs(gm).max()
                assert abs(fd - gm[i, m]) <= tol * scale, (h, i, m, fd, gm[i, m])


def test_grad_wrt_field_by_differences():
    ops, params, d, alpha, sig, tau, th, p, seq, x0, xt = _setup("field")
    L, _, gm = grad.unrolled_loss_and_grad(ops, x0, d, alpha, sig, tau, th, p, seq, xt)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(params.shape)
    h = 1e-6
    lp = grad.unrolled_loss(GatedOperators(12, 14, 18, "field", params + h * v), x0, d, alpha, sig, tau, th, p, seq, xt)
    lm = grad.unrolled_loss(GatedOperators(12, 14, 18, "field", params - h * v), x0, d, alpha, sig, tau, th, p, seq, xt)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - float(np.sum(gm * v))) < 1e-4 * max(1.0, abs(fd))
