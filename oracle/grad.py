"""Gradient through unrolled SPDHG iterations (FP64), by the transposed
iteration map.

The loss is L = |x^K - x_target|^2 after K iterations of Algorithm 1 started
from (x^0, y = 0, z = 0, z-bar = 0) with fixed data d_i. Its gradient is taken
with respect to the starting image x^0 and the motion parameters of every gate
(rigid: (phi, t_x, t_y); field: u_x, u_y at every pixel). D_i(theta) enters
each iteration twice, in A_i = A D_i and in A_i^* = D_i^T A^T; the derivative
of the bilinear interpolant takes the branch of floor() at grid lines.

One iteration, gate i, and its reverse:
  x1 = c_x (x - tau zbar)            c_x = 1 / (1 + 2 tau alpha)
  s  = A D_i x1
  y1 = c_y (y_i + sigma_i (s - d_i)) c_y = 1 / (1 + sigma_i N / 2)
  dy = y1 - y_i,  b = A^T dy,  dz = D_i^T b
  z1 = z + dz,    zbar1 = z1 + (theta / p_i) dz
"""
from __future__ import annotations

import numpy as np

from . import warp
from .operators import GatedOperators
from .spdhg import State, iterate


def _motion_grad(ops: GatedOperators, i, h, v):
    """d/d(motion of gate i) of <h, D_i v>."""
    px, py = ops.pos[i]
    gx, gy = warp.warp_gradient_at(v, px, py)
    if ops.kind == "rigid":
        out = np.zeros(3)
        for m, (dpx, dpy) in enumerate(warp.rigid_position_derivs(ops.n, ops.params[i][0])):
            out[m] = float(np.sum(h * (gx * dpx + gy * dpy)))
        return out
    if ops.kind == "field":
        return np.stack([h * gx, h * gy])
    return None


def unrolled_loss_and_grad(ops: GatedOperators, x0, d, alpha, sigma, tau, theta, p,
                           gate_seq, x_target):
    """Returns (L, dL/dx0, dL/dmotion) with dL/dmotion shaped like ops.params."""
    N = ops.n_gates
    n, na, nd = ops.n, ops.n_angles, ops.n_det
    st = State(np.asarray(x0, dtype=np.float64).copy(),
               [np.zeros((na, nd)) for _ in range(N)], np.zeros((n, n)), np.zeros((n, n)))
    states = [st]
    for i in gate_seq:
        st = iterate(ops, st, d, alpha, sigma, tau, theta, p, [int(i)])
        states.append(st)
    resid = states[-1].x - x_target
    loss = float(np.sum(resid ** 2))

    gx = 2.0 * resid
    gy = [np.zeros((na, nd)) for _ in range(N)]
    gz = np.zeros((n, n))
    gzb = np.zeros((n, n))
    gmot = None if ops.params is None else np.zeros_like(ops.params)
    cx = 1.0 / (1.0 + 2.0 * tau * alpha)
    for k in range(len(gate_seq) - 1, -1, -1):
        i = int(gate_seq[k])
        prev = states[k]
        cy = 1.0 / (1.0 + sigma[i] * N / 2.0)
        # recompute the forward quantities of iteration k
        x1 = cx * (prev.x - tau * prev.zbar)
        s = ops.A(i, x1)
        y1 = cy * (prev.y[i] + sigma[i] * (s - d[i]))
        b = ops.backproject(y1 - prev.y[i])
        # reverse of the z / z-bar update
        gdz = gz + (1.0 + theta / p[i]) * gzb
        gz = gz + gzb
        # dz = D_i^T b
        gb = ops.D(i, gdz)
        if gmot is not None:
            gmot[i] += _motion_grad(ops, i, b, gdz)
        # b = A^T dy ; dy = y1 - y_i ; y1 = c_y (y_i + sigma (s - d))
        gdy = ops.project(gb)
        big_g = gy[i] + gdy
        gy[i] = cy * big_g - gdy
        gs = cy * sigma[i] * big_g
        # s = A D_i x1
        gw = ops.backproject(gs)
        gx1 = gx + ops.Dt(i, gw)
        if gmot is not None:
            gmot[i] += _motion_grad(ops, i, gw, x1)
        # x1 = c_x (x - tau zbar)
        gx = cx * gx1
        gzb = -tau * cx * gx1
    return loss, gx, gmot


def unrolled_loss(ops: GatedOperators, x0, d, alpha, sigma, tau, theta, p, gate_seq, x_target):
    """L alone (for finite differences)."""
    N = ops.n_gates
    n, na, nd = ops.n, ops.n_angles, ops.n_det
    st = State(np.asarray(x0, dtype=np.float64).copy(),
               [np.zeros((na, nd)) for _ in range(N)], np.zeros((n, n)), np.zeros((n, n)))
    for i in gate_seq:
        st = iterate(ops, st, d, alpha, sigma, tau, theta, p, [int(i)])
    return float(np.sum((st.x - x_target) ** 2))
