"""SPDHG sampling over gates x angle subsets, in FP64 (test infrastructure).

The Conclusions name sampling over both the gates and subsets of the data
(e.g. angles) as the next step. This module is that extension of Algorithm 1,
written from the model of Section II-A:

* the angles are cut into M subsets, either contiguous ranges
  [k_s, k_{s+1}) with k_s = floor(s n_a / M), or (n_a even) paired ranges
  [h_s, h_{s+1}) and [h_s + n_a/2, h_{s+1} + n_a/2) with h_s = floor(s n_a / (2M)),
  every angle together with the one a quarter turn away (the Conclusions
  name no partition; any partition of the angles gives the same problem);
  R_s keeps the sinogram rows of subset s;
* a block b = (i, s) (b = i M + s) has the operator A_b = R_s A D_i and the
  data term f_b(u) = |u - d_{i,s}|^2 / N, so that sum_s f_{(i,s)}(R_s u) equals
  the gate's f_i(u): the objective O, its minimiser x* and the dual solution
  (y*_{i,s} = R_s y*_i) are those of the gate problem;
* f_b^* has the same strong convexity modulus N/2 as f_i^*, so block b's
  condition number is |A_b|^2 / (alpha N) and its proximal map is the gate
  formula restricted to the block's rows;
* Algorithm 1 runs over the N M blocks with probabilities p_b (serial uniform
  sampling: p_b = 1 / (N M)); an epoch is N M block iterations, the same
  number of projector applications as one PDHG iteration.

The dual variables stay per gate (full [n_a][n_d] arrays); a block reads and
writes only its subset's rows. This is plain, slow reference code: a block
operator projects the whole sinogram and masks it.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from . import spdhg


def subset_bounds(n_angles: int, n_subsets: int):
    """k_0 = 0 < k_1 < ... < k_M = n_angles with k_s = floor(s n_angles / M)."""
    if not 1 <= n_subsets <= n_angles:
        raise ValueError("need 1 <= n_subsets <= n_angles")
    return [(s * n_angles) // n_subsets for s in range(n_subsets + 1)]


def contiguous_subsets(n_angles: int, n_subsets: int):
    """Subset s = the angles [k_s, k_{s+1}) (index arrays)."""
    kb = subset_bounds(n_angles, n_subsets)
    return [np.arange(kb[s], kb[s + 1]) for s in range(n_subsets)]


def paired_subsets(n_angles: int, n_subsets: int):
    """Subset s = the angles [h_s, h_{s+1}) and their partners a quarter turn
    away, [h_s + n_a/2, h_{s+1} + n_a/2), h_s = floor(s (n_a/2) / M) (n_a even,
    1 <= M <= n_a/2)."""
    if n_angles % 2:
        raise ValueError("paired subsets need an even number of angles")
    half = n_angles // 2
    hb = subset_bounds(half, n_subsets)
    return [np.concatenate([np.arange(hb[s], hb[s + 1]), np.arange(hb[s] + half, hb[s + 1] + half)])
            for s in range(n_subsets)]


class BlockOperators:
    """Blocks b = i M + s of a GatedOperators `ops` and M angle subsets.

    partition: "contiguous" (default), "paired", or an explicit list of M
    index arrays that together hold every angle exactly once."""

    def __init__(self, ops, n_subsets: int, partition="contiguous"):
        self.ops = ops
        self.n_gates = ops.n_gates
        self.n_subsets = int(n_subsets)
        self.n_blocks = self.n_gates * self.n_subsets
        self.n, self.n_angles, self.n_det = ops.n, ops.n_angles, ops.n_det
        if isinstance(partition, str):
            make = {"contiguous": contiguous_subsets, "paired": paired_subsets}[partition]
            parts = make(ops.n_angles, self.n_subsets)
        else:
            parts = [np.sort(np.asarray(p, dtype=np.int64)) for p in partition]
        if len(parts) != self.n_subsets:
            raise ValueError("the partition needs one index array per subset")
        seen = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
        if not np.array_equal(np.sort(seen), np.arange(ops.n_angles)):
            raise ValueError("the subsets must hold every angle exactly once")
        self.parts = parts

    def split(self, b: int):
        """(gate, subset) of block b."""
        return divmod(int(b), self.n_subsets)

    def rows(self, s: int) -> np.ndarray:
        """The sinogram rows (angles) of subset s."""
        return self.parts[s]

    def mask(self, s: int, y):
        """R_s^T R_s y: the rows of subset s, zero elsewhere."""
        out = np.zeros_like(np.asarray(y, dtype=np.float64))
        out[self.rows(s)] = np.asarray(y, dtype=np.float64)[self.rows(s)]
        return out

    def A(self, b, x):
        """A_b x as a full-size sinogram, zero outside the block's rows."""
        i, s = self.split(b)
        return self.mask(s, self.ops.A(i, x))

    def At(self, b, y):
        """A_b^* y = D_i^T A^T R_s^T R_s y."""
        i, s = self.split(b)
        return self.ops.At(i, self.mask(s, y))


def iterate(bops: BlockOperators, state: spdhg.State, d, alpha, sigma, tau, theta, p,
            S: Sequence[int]) -> spdhg.State:
    """One iteration of Algorithm 1 over blocks (returns a new state).

    (i)   x <- prox_{tau g}(x - tau z-bar)
    (ii)  for b = (i, s) in S: the rows of subset s of y_i become
          prox_{sigma_b f_b^*}(y_{i,s} + sigma_b A_b x), with the gate count N
          in the proximal map (f_b keeps the 1/N of f_i)
    (iii) z <- z + sum_{b in S} A_b^*(y_b' - y_b);
          z-bar <- z_new + sum_{b in S} (theta / p_b) A_b^*(y_b' - y_b)
    """
    N = bops.n_gates
    x = spdhg.prox_tau_g(state.x - tau * state.zbar, tau, alpha)
    y = [v.copy() for v in state.y]
    dz = np.zeros_like(state.z)
    dzbar = np.zeros_like(state.z)
    for b in S:
        i, s = bops.split(b)
        r = bops.rows(s)
        old = y[i][r].copy()
        ax = bops.A(b, x)[r]
        y[i][r] = spdhg.prox_sigma_fstar(old + sigma[b] * ax, sigma[b], np.asarray(d[i])[r], N)
        diff = np.zeros_like(y[i])
        diff[r] = y[i][r] - old
        delta = bops.At(b, diff)
        dz += delta
        dzbar += (theta / p[b]) * delta
    z = state.z + dz
    return spdhg.State(x, y, z, z + dzbar)


def spdhg_blocks(bops, state, d, alpha, sigma, tau, theta, p, block_seq) -> spdhg.State:
    """Serial sampling: one block per iteration, the blocks given by `block_seq`."""
    for b in block_seq:
        state = iterate(bops, state, d, alpha, sigma, tau, theta, p, [int(b)])
    return state


def block_norm_sq(bops, b, v0, **kw):
    """|A_b|^2 by power iteration on A_b^* A_b."""
    return spdhg.power_norm_sq(lambda v: bops.At(b, bops.A(b, v)), v0, **kw)


def step_sizes(norms_sq_blocks, alpha, n_gates):
    """Step sizes for serial uniform sampling over the blocks (p = 1/(N M)),
    the rule of the gate case with the block norms: s_b = sqrt(1 + kappa_b),
    kappa_b = |A_b|^2 / (alpha N), s = max s_b, rho = 1 - 2p/(1 + s),
    sigma_b = 2/(N (s_b - 1)), tau = p/(2 alpha rho (1 + s)), theta = rho.
    Returns (sigma[NM], tau, theta, rho) with rho the per-iteration rate; the
    per-epoch rate is rho^(N M) = l(max kappa_b, N M)."""
    nb = len(norms_sq_blocks)
    pr = 1.0 / nb
    s_b = [math.sqrt(1.0 + a / (alpha * n_gates)) for a in norms_sq_blocks]
    s = max(s_b)
    rho = 1.0 - 2.0 * pr / (1.0 + s)
    sigma = [2.0 / (n_gates * (sb - 1.0)) for sb in s_b]
    tau = pr / (2.0 * alpha * rho * (1.0 + s))
    return sigma, tau, rho, rho


def epoch_rate(norms_sq_blocks, alpha, n_gates):
    """Per-epoch rate l(kappa, N M) with kappa = max_b |A_b|^2 / (alpha N)."""
    return spdhg.rate(max(norms_sq_blocks) / (alpha * n_gates), len(norms_sq_blocks))

