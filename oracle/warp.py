"""Displacement operator D_i: X -> X (Section II-A) and its transpose (FP64).

D_i is read as the pull-back of the image through the gate's motion map,
(D_i x)(p) = x~(phi_i(p)), where x~ is the bilinear interpolant of x with zero
outside the image, in index coordinates (x = column, y = row). The paper's two
kinds of motion (Section III, "Description"):

* rigid (rotation and translation): phi(p) = R(phi) (p - c) + c + t with
  c = ((n-1)/2, (n-1)/2), parameters (phi [rad], t_x, t_y [px]);
* non-rigid: phi(p) = p + u(p) for a displacement field u = (u_x, u_y).

D_i^T is the scatter of exactly the same bilinear weights, so it is the exact
transpose of `warp` by construction (Algorithm 1 step (iii) uses
A_i^* = D_i^* A^*).
"""
from __future__ import annotations

import numpy as np


def rigid_positions(n: int, phi: float, tx: float, ty: float):
    """Sample positions (column, row) of every output pixel under rigid motion."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    x -= c
    y -= c
    cp, sp = np.cos(phi), np.sin(phi)
    px = cp * x - sp * y + c + tx
    py = sp * x + cp * y + c + ty
    return px, py


def rigid_position_derivs(n: int, phi: float):
    """d(px, py)/d(phi, t_x, t_y) at every pixel: three pairs of [n][n] arrays."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    x -= c
    y -= c
    cp, sp = np.cos(phi), np.sin(phi)
    one, zero = np.ones((n, n)), np.zeros((n, n))
    return [(-sp * x - cp * y, cp * x - sp * y), (one, zero), (zero, one)]


def field_positions(u: np.ndarray):
    """Sample positions (column, row) = p + u(p) for a field u [2][n][n]."""
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[-1]
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return x + u[0], y + u[1]


def _taps(px, py):
    c0 = np.floor(px)
    r0 = np.floor(py)
    fx = px - c0
    fy = py - r0
    c0 = c0.astype(np.int64)
    r0 = r0.astype(np.int64)
    return [(r0, c0, (1 - fx) * (1 - fy)), (r0, c0 + 1, fx * (1 - fy)),
            (r0 + 1, c0, (1 - fx) * fy), (r0 + 1, c0 + 1, fx * fy)]


def warp(x: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """D x: bilinear samples of x at (px, py), zero outside the image."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    out = np.zeros((n, n))
    for rr, cc, w in _taps(px, py):
        ok = (rr >= 0) & (rr < n) & (cc >= 0) & (cc < n)
        out += np.where(ok, w * x[np.clip(rr, 0, n - 1), np.clip(cc, 0, n - 1)], 0.0)
    return out


def warp_adjoint(b: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """D^T b: every output pixel p sends b(p) times its bilinear weights back to
    the taps it read."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    acc = np.zeros(n * n)
    for rr, cc, w in _taps(px, py):
        ok = (rr >= 0) & (rr < n) & (cc >= 0) & (cc < n)
        acc += np.bincount((rr * n + cc)[ok], weights=(w * b)[ok], minlength=n * n)
    return acc.reshape(n, n)


def warp_gradient_at(v: np.ndarray, px: np.ndarray, py: np.ndarray):
    """Spatial gradient (d/dpx, d/dpy) of the bilinear interpolant of v at the
    sample positions, taking the branch of floor() (one-sided at grid lines)."""
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[0]
    c0 = np.floor(px)
    r0 = np.floor(py)
    fx = px - c0
    fy = py - r0
    c0 = c0.astype(np.int64)
    r0 = r0.astype(np.int64)

    def val(rr, cc):
        ok = (rr >= 0) & (rr < n) & (cc >= 0) & (cc < n)
        return np.where(ok, v[np.clip(rr, 0, n - 1), np.clip(cc, 0, n - 1)], 0.0)

    v00, v01 = val(r0, c0), val(r0, c0 + 1)
    v10, v11 = val(r0 + 1, c0), val(r0 + 1, c0 + 1)
    gx = (1 - fy) * (v01 - v00) + fy * (v11 - v10)
    gy = (1 - fx) * (v10 - v00) + fx * (v11 - v01)
    return gx, gy
