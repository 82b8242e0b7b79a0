"""Algorithm 1 (SPDHG, with PDHG as a special case) and its theory, in FP64.

Model (Section II-A): minimise O(x) = g(x) + sum_i f_i(A_i x) with
f_i(u) = |u - d_i|^2 / N and g(x) = alpha |x|^2. Derived from these:

* f_i^*(y) = <y, d_i> + (N/4) |y|^2,  prox_{s f_i^*}(v) = (v - s d_i) / (1 + s N / 2);
* g^*(w) = |w|^2 / (4 alpha),         prox_{t g}(v)     = v / (1 + 2 t alpha);
* strong convexity moduli 2 alpha (g) and N/2 (f_i^*), so the condition number
  of gate i is |A_i|^2 / (alpha N), as in Theorem 1.

Algorithm 1 is read with the extrapolated dual image in step (i) and the
extrapolation of step (iii) taken from z (the printed z-bar recursion does not
converge).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np


# ----------------------------------------------------------------------------
# Proximal maps (Algorithm 1, steps (i) and (ii))
# ----------------------------------------------------------------------------
def prox_tau_g(v, tau, alpha):
    """prox of tau * alpha |.|^2."""
    return v / (1.0 + 2.0 * tau * alpha)


def prox_sigma_fstar(v, sigma, d, n_gates):
    """prox of sigma * f_i^* with f_i(u) = |u - d|^2 / N."""
    return (v - sigma * d) / (1.0 + sigma * n_gates / 2.0)


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    """(x, y_1..y_N, z, z-bar) of Algorithm 1; all zero at initialisation."""
    x: np.ndarray
    y: list
    z: np.ndarray
    zbar: np.ndarray

    @staticmethod
    def zeros(n, n_gates, n_angles, n_det):
        return State(np.zeros((n, n)), [np.zeros((n_angles, n_det)) for _ in range(n_gates)],
                     np.zeros((n, n)), np.zeros((n, n)))

    def copy(self):
        return State(self.x.copy(), [v.copy() for v in self.y], self.z.copy(), self.zbar.copy())


def iterate(ops, state: State, d, alpha, sigma, tau, theta, p, S: Sequence[int]) -> State:
    """One iteration of Algorithm 1 with the drawn gate set S (returns a new state).

    (i)   x <- prox_{tau g}(x - tau z-bar)
    (ii)  y_i <- prox_{sigma_i f_i^*}(y_i + sigma_i A_i x) for i in S
    (iii) z <- z + sum_{i in S} A_i^*(y_i' - y_i);
          z-bar <- z_new + sum_{i in S} (theta / p_i) A_i^*(y_i' - y_i)
    """
    N = ops.n_gates
    x = prox_tau_g(state.x - tau * state.zbar, tau, alpha)
    y = list(state.y)
    dz = np.zeros_like(state.z)
    dzbar = np.zeros_like(state.z)
    for i in S:
        yi = prox_sigma_fstar(state.y[i] + sigma[i] * ops.A(i, x), sigma[i], d[i], N)
        delta = ops.At(i, yi - state.y[i])
        dz += delta
        dzbar += (theta / p[i]) * delta
        y[i] = yi
    z = state.z + dz
    return State(x, y, z, z + dzbar)


def spdhg(ops, state: State, d, alpha, sigma, tau, theta, p, gate_seq) -> State:
    """SPDHG: one gate per iteration, the gates given by `gate_seq` (serial sampling)."""
    for i in gate_seq:
        state = iterate(ops, state, d, alpha, sigma, tau, theta, p, [int(i)])
    return state


def pdhg(ops, state: State, d, alpha, sigma, tau, theta, iters: int = 1) -> State:
    """PDHG: every gate every iteration with p_i = 1 (Section II-A)."""
    ones = [1.0] * ops.n_gates
    for _ in range(iters):
        state = iterate(ops, state, d, alpha, sigma, tau, theta, ones, list(range(ops.n_gates)))
    return state


# ----------------------------------------------------------------------------
# Rates and step sizes (Section II-B, Theorem 1)
# ----------------------------------------------------------------------------
def rate(kappa, n):
    """l(kappa, n) = (1 - 2 / (n (1 + sqrt(1 + kappa))))^n."""
    return (1.0 - 2.0 / (n * (1.0 + math.sqrt(1.0 + kappa)))) ** n


def condition_numbers(norms_sq_gates, norm_sq_stacked, alpha, n_gates):
    """Theorem 1: kappa^SPDHG = max_i |A_i|^2 / (alpha N), kappa^PDHG = |(A_1..A_N)|^2 / (alpha N)."""
    return max(norms_sq_gates) / (alpha * n_gates), norm_sq_stacked / (alpha * n_gates)


def step_sizes_spdhg(norms_sq_gates, alpha, n_gates):
    """Step sizes for serial uniform sampling (p = 1/N) that attain the per-epoch
    rate l(kappa^SPDHG, N) of Theorem 1. Returns (sigma[N], tau, theta, rho)
    with rho the per-iteration rate."""
    N = n_gates
    pr = 1.0 / N
    s_i = [math.sqrt(1.0 + a / (alpha * N)) for a in norms_sq_gates]
    s = max(s_i)
    rho = 1.0 - 2.0 * pr / (1.0 + s)
    sigma = [2.0 / (N * (si - 1.0)) for si in s_i]
    tau = pr / (2.0 * alpha * rho * (1.0 + s))
    return sigma, tau, rho, rho


def step_sizes_pdhg(norm_sq_stacked, alpha, n_gates):
    """Step sizes of accelerated PDHG that attain the per-epoch rate l(kappa^PDHG, 1)."""
    N = n_gates
    s = math.sqrt(1.0 + norm_sq_stacked / (alpha * N))
    rho = (s - 1.0) / (s + 1.0)
    sigma = [2.0 / (N * (s - 1.0))] * N
    tau = 1.0 / (2.0 * alpha * (s - 1.0))
    return sigma, tau, rho, rho


# ----------------------------------------------------------------------------
# Norms by power iteration (Theorem 1 needs |A_i|^2 and |(A_1..A_N)|^2)
# ----------------------------------------------------------------------------
def power_norm_sq(apply_normal, v0, rtol=1e-12, max_iter=500):
    """Largest eigenvalue of the symmetric PSD map `apply_normal` (A^* A) by power
    iteration from v0; stops when the Rayleigh quotient changes by less than rtol
    (relative). Returns (lambda, iterations)."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for it in range(1, max_iter + 1):
        w = apply_normal(v)
        lam_new = float(np.vdot(v, w))
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0, it
        v = w / nw
        if it > 1 and abs(lam_new - lam) <= rtol * abs(lam_new):
            return lam_new, it
        lam = lam_new
    return lam, max_iter


def gate_norm_sq(ops, i, v0, **kw):
    return power_norm_sq(lambda v: ops.At(i, ops.A(i, v)), v0, **kw)


def stacked_norm_sq(ops, v0, **kw):
    return power_norm_sq(lambda v: sum(ops.At(i, ops.A(i, v)) for i in range(ops.n_gates)), v0, **kw)


# ----------------------------------------------------------------------------
# Saddle point, objective, gap, distance
# ----------------------------------------------------------------------------
def saddle_point(ops, d, alpha, rtol=1e-13, max_iter=5000, dense=False):
    """x* = (alpha I + N^-1 sum A_i^* A_i)^-1 N^-1 sum A_i^* d_i, the unique
    minimiser of O; y_i* = (2/N)(A_i x* - d_i) (the optimality condition of
    f_i). Dense solve for tiny sizes, else conjugate gradients."""
    N = ops.n_gates
    n = ops.n
    rhs = sum(ops.At(i, d[i]) for i in range(N)) / N

    def normal(v):
        return alpha * v + sum(ops.At(i, ops.A(i, v)) for i in range(N)) / N

    if dense:
        m = np.zeros((n * n, n * n))
        e = np.zeros(n * n)
        for q in range(n * n):
            e[:] = 0.0
            e[q] = 1.0
            m[:, q] = normal(e.reshape(n, n)).ravel()
        xs = np.linalg.solve(m, rhs.ravel()).reshape(n, n)
    else:
        xs = np.zeros((n, n))
        r = rhs - normal(xs)
        pdir = r.copy()
        rr = float(np.vdot(r, r))
        b2 = float(np.vdot(rhs, rhs))
        for _ in range(max_iter):
            ap = normal(pdir)
            a = rr / float(np.vdot(pdir, ap))
            xs = xs + a * pdir
            r = r - a * ap
            rr_new = float(np.vdot(r, r))
            if rr_new <= (rtol ** 2) * b2:
                break
            pdir = r + (rr_new / rr) * pdir
            rr = rr_new
    ys = [(2.0 / N) * (ops.A(i, xs) - d[i]) for i in range(N)]
    return xs, ys


def objective(ops, x, d, alpha):
    """O(x) = alpha |x|^2 + N^-1 sum_i |A_i x - d_i|^2."""
    N = ops.n_gates
    return alpha * float(np.vdot(x, x)) + sum(float(np.sum((ops.A(i, x) - d[i]) ** 2)) for i in range(N)) / N


def duality_gap(ops, x, y, d, alpha):
    """O(x) + g^*(-z) + sum_i f_i^*(y_i) with z = sum_i A_i^* y_i (>= 0, zero only
    at the saddle point)."""
    N = ops.n_gates
    z = sum(ops.At(i, y[i]) for i in range(N))
    dual = float(np.vdot(z, z)) / (4.0 * alpha) + sum(
        float(np.vdot(y[i], d[i])) + 0.25 * N * float(np.vdot(y[i], y[i])) for i in range(N))
    return objective(ops, x, d, alpha) + dual


def dist_sq(state: State, xs, ys):
    """|x - x*|^2 + sum_i |y_i - y_i*|^2 (the distance plotted in Fig. 1)."""
    return float(np.sum((state.x - xs) ** 2)) + sum(float(np.sum((a - b) ** 2)) for a, b in zip(state.y, ys))


def make_data(ops, x_true, unit_noise, rel_noise=0.01):
    """d_i = A_i x + eps_i, eps_i ~ N(0, s^2 / N) per entry with
    s = rel_noise * max|A x| (Section II-A; the un-warped image sets the scale)."""
    N = ops.n_gates
    scale = rel_noise * float(np.max(np.abs(ops.project(x_true))))
    return [ops.A(i, x_true) + (scale / math.sqrt(N)) * unit_noise[i] for i in range(N)]
