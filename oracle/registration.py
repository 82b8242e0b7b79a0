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

    s = np.asarray(theta0, dtype=np.float64) * scale
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
    return s / scale, E, k
