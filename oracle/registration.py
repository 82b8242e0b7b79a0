"""Rigid registration of a gated image to the reference image (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section I places the estimation of the displacement maps, from the reference
motion state to every gate, in a preliminary step before the reconstruction,
and does not say how it is done. This module takes the following reading,
for the rigid motion of Section III ("Description"): the parameters
theta = (phi, t_x, t_y) of gate i minimise the squared misfit

    E(theta) = 1/2 |D(theta) ref - target|^2,

with D(theta) the bilinear pull-back of `warp` (zero outside the image), ref
the reference-state image and target the gate's image. Its gradient is
J^T (D(theta) ref - target), J the derivative of D(theta) ref with respect to
theta (the chain rule through the sample positions, the floor branch of the
bilinear interpolant at grid lines).

The minimisation is gradient descent in the scaled coordinates
s = (phi (n - 1) / 2, t_x, t_y), in which every coordinate is a displacement
in pixels at the image's edge, with Barzilai-Borwein step lengths (the first
trial moves 1 px) and Armijo backtracking (sufficient decrease 1e-4, step
halved at most 40 times). It stops after the first accepted step shorter than
`tol` pixels, at a zero gradient, or after `max_iter` steps.

The chest experiment's non-rigid motion is a linear dilatation (Section III),
an affine map. `register_affine` takes the displacement field
u(p) = A (p - c) + t (x = column - c, y = row - c, c = (n - 1) / 2), six
parameters (A00, A01, A10, A11, t_x, t_y), rounded to float32 per pixel as
the library stores fields, with the same minimisation in the scaled
coordinates (A (n - 1) / 2, t).

`register_field` estimates a dense displacement field u [2][n][n] (the
displacement maps of Section II-A themselves). The reading: u minimises

    E(u) = 1/2 |D_u ref - target|^2 + lambda / 2 R(u),

R(u) the sum, over both components, of the squared differences between
horizontally and vertically adjacent pixels of the image (a discrete
Dirichlet energy; pixels outside the image take no part). Its gradient is
r * grad(ref)(p + u(p)) + lambda L u, r the residual and (L u)(p) the sum of
u(p) - u(q) over the image neighbours q of p. The field is stored in
float32, so E and its gradient are evaluated on the float32-rounded field;
the iterate itself is kept in float64. The minimisation is the same
Barzilai-Borwein / Armijo descent, directly in the field's pixel units, with
`tol` bounding the Euclidean norm of the whole accepted step.

A single level of that descent converges slowly when the images are smooth
or piecewise constant and the displacement spans several pixels. The
reading adds a scale-space schedule: for each width sigma of a given list
(pixels, decreasing; 0 = no smoothing) both images are smoothed with the
separable Gaussian of that width (weights exp(-k^2 / (2 sigma^2)) for
|k| <= int(3 sigma + 0.5), normalised to sum 1, zero outside the image) and
the descent runs from the previous level's field.
"""
from __future__ import annotations

import numpy as np

from . import warp


def energy_and_grad(ref: np.ndarray, target: np.ndarray, theta) -> tuple[float, np.ndarray]:
    """E(theta) and dE/dtheta (phi, t_x, t_y) for 2D float64 images."""
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[0]
    px, py = warp.rigid_positions(n, float(theta[0]), float(theta[1]), float(theta[2]))
    r = warp.warp(ref, px, py) - np.asarray(target, dtype=np.float64)
    gx, gy = warp.warp_gradient_at(ref, px, py)
    g = np.array([float(np.sum(r * (gx * dpx + gy * dpy)))
                  for dpx, dpy in warp.rigid_position_derivs(n, float(theta[0]))])
    return 0.5 * float(np.sum(r * r)), g


def register_rigid(ref, target, theta0=(0.0, 0.0, 0.0), max_iter: int = 200, tol: float = 1e-6):
    """Returns (theta, E(theta), steps taken)."""
    n = np.asarray(ref).shape[0]
    rad = (n - 1) / 2.0
    scale = np.array([rad, 1.0, 1.0])

    def ev(s):
        E, g = energy_and_grad(ref, target, s / scale)
        return E, g / scale  # gradient with respect to the scaled coordinates

    s, E, k = _minimise(ev, np.asarray(theta0, dtype=np.float64) * scale, max_iter, tol)
    return s / scale, E, k


def affine_field(n: int, theta) -> np.ndarray:
    """u [2][n][n] of the affine map theta = (A00, A01, A10, A11, t_x, t_y),
    each component evaluated as (A_r0 x + A_r1 y) + t_r in float64 and rounded
    to float32."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    x -= c
    y -= c
    a00, a01, a10, a11, tx, ty = (float(v) for v in theta)
    u = np.stack([(a00 * x + a01 * y) + tx, (a10 * x + a11 * y) + ty])
    return u.astype(np.float32).astype(np.float64)


def energy_and_grad_affine(ref: np.ndarray, target: np.ndarray, theta) -> tuple[float, np.ndarray]:
    """E(theta) and dE/dtheta for the affine displacement field."""
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[0]
    px, py = warp.field_positions(affine_field(n, theta))
    r = warp.warp(ref, px, py) - np.asarray(target, dtype=np.float64)
    gx, gy = warp.warp_gradient_at(ref, px, py)
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    xx -= c
    yy -= c
    hx, hy = r * gx, r * gy
    g = np.array([np.sum(hx * xx), np.sum(hx * yy), np.sum(hy * xx), np.sum(hy * yy), np.sum(hx), np.sum(hy)])
    return 0.5 * float(np.sum(r * r)), g


def _minimise(ev, s, max_iter, tol):
    """Gradient descent with Barzilai-Borwein steps and Armijo backtracking on
    the scaled coordinates s (see the module docstring)."""
    E, g = ev(s)
    gn = float(np.linalg.norm(g))
    alpha = 1.0 / gn if gn > 0 else 1.0
    k = 0
    while k < max_iter and gn > 0:
        for _ in range(41):
            s_new = s - alpha * g
            E_new, g_new = ev(s_new)
            if E_new <= E - 1e-4 * alpha * gn * gn:
                break
            alpha *= 0.5
        k += 1
        step = alpha * gn
        ds, dg = s_new - s, g_new - g
        s, E, g = s_new, E_new, g_new
        gn = float(np.linalg.norm(g))
        if step < tol:
            break
        sy = float(ds @ dg)
        alpha = float(ds @ ds) / sy if sy > 0 else 2.0 * alpha
    return s, E, k


def register_affine(ref, target, theta0=(0.0,) * 6, max_iter: int = 300, tol: float = 1e-6):
    """Returns (theta, E(theta), steps taken) for the affine displacement field."""
    n = np.asarray(ref).shape[0]
    rad = (n - 1) / 2.0
    scale = np.array([rad, rad, rad, rad, 1.0, 1.0])

    def ev(s):
        E, g = energy_and_grad_affine(ref, target, s / scale)
        return E, g / scale

    s, E, k = _minimise(ev, np.asarray(theta0, dtype=np.float64) * scale, max_iter, tol)
    return s / scale, E, k


def field_regulariser(u) -> tuple[float, np.ndarray]:
    """R(u) (see the module docstring) and L u, for u [2][n][n]."""
    u = np.asarray(u, dtype=np.float64)
    dx = np.diff(u, axis=2)  # u(r, c + 1) - u(r, c)
    dy = np.diff(u, axis=1)  # u(r + 1, c) - u(r, c)
    R = float(np.sum(dx * dx) + np.sum(dy * dy))
    Lu = np.zeros_like(u)
    Lu[:, :, :-1] -= dx
    Lu[:, :, 1:] += dx
    Lu[:, :-1, :] -= dy
    Lu[:, 1:, :] += dy
    return R, Lu


def energy_and_grad_field(ref, target, u, lam: float, round32: bool = True) -> tuple[float, np.ndarray]:
    """E(u) and dE/du [2][n][n] for the dense displacement field (evaluated on
    the float32-rounded field unless round32 is False)."""
    ref = np.asarray(ref, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    ue = u.astype(np.float32).astype(np.float64) if round32 else u
    px, py = warp.field_positions(ue)
    r = warp.warp(ref, px, py) - np.asarray(target, dtype=np.float64)
    gx, gy = warp.warp_gradient_at(ref, px, py)
    R, Lu = field_regulariser(ue)
    E = 0.5 * float(np.sum(r * r)) + 0.5 * lam * R
    return E, np.stack([r * gx, r * gy]) + lam * Lu


def gaussian_smooth(img, sigma: float) -> np.ndarray:
    """The separable Gaussian of width sigma (see the module docstring),
    along columns then rows, zero outside the image; sigma = 0: a copy."""
    img = np.asarray(img, dtype=np.float64)
    if sigma == 0:
        return img.copy()
    R = int(3.0 * sigma + 0.5)
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    w /= w.sum()
    n = img.shape[0]
    out = img
    for axis in (1, 0):
        acc = np.zeros_like(out)
        for j, wj in zip(range(-R, R + 1), w):
            # acc[p] += w_j * out[p + j e_axis], zero outside the image
            src = [slice(None), slice(None)]
            dst = [slice(None), slice(None)]
            if j >= 0:
                src[axis], dst[axis] = slice(j, n), slice(0, n - j)
            else:
                src[axis], dst[axis] = slice(0, n + j), slice(-j, n)
            acc[tuple(dst)] += wj * out[tuple(src)]
        out = acc
    return out


def register_field(ref, target, u0=None, lam: float = 0.1, max_iter: int = 200, tol: float = 1e-3,
                   sigmas=()):
    """Returns (u [2][n][n] float64, E(u) of the last level, steps taken over
    all levels) for the dense field, started from u0 (default zero); sigmas:
    the scale-space schedule (empty: one level on the images themselves),
    max_iter and tol per level."""
    n = np.asarray(ref).shape[0]
    shape = (2, n, n)
    s = (np.zeros(shape) if u0 is None else np.asarray(u0, dtype=np.float64)).ravel().copy()
    E, k_total = 0.0, 0
    for sigma in (tuple(sigmas) or (0.0,)):
        rs, ts = gaussian_smooth(ref, sigma), gaussian_smooth(target, sigma)

        def ev(v, rs=rs, ts=ts):
            Ev, g = energy_and_grad_field(rs, ts, v.reshape(shape), lam)
            return Ev, g.ravel()

        s, E, k = _minimise(ev, s, max_iter, tol)
        k_total += k
    return s.reshape(shape), E, k_total
