"""Pins of the oracle's Algorithm 1 and its theory: proximal optimality,
invariants, the saddle point as a linear solve, power iteration against a
library SVD, the closed forms of l(kappa, n), the exact spectral radius of the
iteration on tiny problems, and the observed rates in the paper's regime
(kappa ~ 70, Section III)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import spdhg, projector
from oracle.operators import GatedOperators
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class MatrixOps:
    """Explicit-matrix gate operators for the spectral tests."""

    def __init__(self, mats):
        self.mats = [np.asarray(m, dtype=np.float64) for m in mats]
        self.n_gates = len(mats)

    def A(self, i, x):
        return self.mats[i] @ x

    def At(self, i, y):
        return self.mats[i].T @ y


def small_problem(n=16, na=18, nd=24, N=3, alpha=5.0, seed=0):
    ops = GatedOperators(n, na, nd, "rigid", synth.rigid_params(N, seed + 1, 6.0, 2.0))
    x_true = synth.ellipse_phantom(n, seed).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((N, na, nd), seed + 2))
    return ops, d, alpha


def test_prox_optimality():
    rng = np.random.default_rng(0)
    v, d = rng.standard_normal(50), rng.standard_normal(50)
    sig, N, tau, alpha = 0.37, 7, 0.21, 1.9
    y = spdhg.prox_sigma_fstar(v, sig, d, N)
    # y minimises sig f*(y) + |y - v|^2 / 2 with grad f*(y) = d + N y / 2
    np.testing.assert_allclose(y - v + sig * (d + 0.5 * N * y), 0, atol=1e-14)
    x = spdhg.prox_tau_g(v, tau, alpha)
    np.testing.assert_allclose(x - v + tau * 2 * alpha * x, 0, atol=1e-14)


def test_invariant_z_is_sum_of_adjoints():
    ops, d, alpha = small_problem()
    st = spdhg.State.zeros(ops.n, ops.n_gates, ops.n_angles, ops.n_det)
    sigma, tau, theta, _ = spdhg.step_sizes_spdhg([1e3] * 3, alpha, 3)
    st = spdhg.spdhg(ops, st, d, alpha, sigma, tau, theta, [1 / 3] * 3, [2, 0, 0, 1, 2, 1])
    z = sum(ops.At(i, st.y[i]) for i in range(3))
    np.testing.assert_allclose(st.z, z, atol=1e-10 * np.abs(z).max())


def test_saddle_point_is_fixed_point_and_gap_zero():
    ops, d, alpha = small_problem()
    xs, ys = spdhg.saddle_point(ops, d, alpha, dense=True)
    zs = sum(ops.At(i, ys[i]) for i in range(3))
    np.testing.assert_allclose(zs, -2 * alpha * xs, atol=1e-9 * np.abs(xs).max() * alpha)
    st = spdhg.State(xs.copy(), [v.copy() for v in ys], zs.copy(), zs.copy())
    sigma, tau, theta, _ = spdhg.step_sizes_spdhg([1e3] * 3, alpha, 3)
    out = spdhg.spdhg(ops, st, d, alpha, sigma, tau, theta, [1 / 3] * 3, [0, 2, 1])
    assert spdhg.dist_sq(out, xs, ys) < 1e-20 * (1 + float(np.sum(xs ** 2)))
    gap = spdhg.duality_gap(ops, xs, ys, d, alpha)
    assert abs(gap) < 1e-9 * spdhg.objective(ops, xs, d, alpha)


def test_cg_matches_dense_solve():
    ops, d, alpha = small_problem(n=12, na=14, nd=18)
    x1, _ = spdhg.saddle_point(ops, d, alpha, dense=True)
    x2, _ = spdhg.saddle_point(ops, d, alpha)
    np.testing.assert_allclose(x2, x1, atol=1e-9 * np.abs(x1).max())


def test_single_gate_spdhg_equals_pdhg():
    ops = GatedOperators(12, 10, 18, "rigid", synth.rigid_params(1, 3, 5, 2))
    x_true = synth.ellipse_phantom(12, 1).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((1, 10, 18), 4))
    sigma, tau, theta, _ = spdhg.step_sizes_pdhg(300.0, 2.0, 1)
    st0 = spdhg.State.zeros(12, 1, 10, 18)
    a = spdhg.spdhg(ops, st0, d, 2.0, sigma, tau, theta, [1.0], [0] * 5)
    b = spdhg.pdhg(ops, st0, d, 2.0, sigma, tau, theta, iters=5)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.zbar, b.zbar)


def test_power_iteration_matches_svd():
    ops = GatedOperators(12, 14, 18, "rigid", synth.rigid_params(2, 5, 7, 2))
    m = np.stack([projector.matrix(12, 14, 18) @ np.stack(
        [ops.D(i, e.reshape(12, 12)).ravel() for e in np.eye(144)], axis=1) for i in range(2)])
    v0 = synth.random_image(12, 8).astype(np.float64)
    for i in range(2):
        lam, _ = spdhg.gate_norm_sq(ops, i, v0)
        assert abs(lam - np.linalg.norm(m[i], 2) ** 2) < 1e-10 * lam
    lam, _ = spdhg.stacked_norm_sq(ops, v0)
    assert abs(lam - np.linalg.norm(np.concatenate(m, axis=0), 2) ** 2) < 1e-10 * lam


def test_rate_closed_forms_and_paper_claim():
    # n = 1: l = (s - 1)/(s + 1) with s = sqrt(1 + kappa)
    for kappa in [0.5, 10, 70, 1e4]:
        s = math.sqrt(1 + kappa)
        assert abs(spdhg.rate(kappa, 1) - (s - 1) / (s + 1)) < 1e-15
        # large n: l -> exp(-2 / (1 + s))
        assert abs(spdhg.rate(kappa, 10 ** 7) - math.exp(-2 / (1 + s))) < 1e-6
    # Section II-B: for kappa >= 10, l(kappa / N, N) < l(kappa, 1)
    for kappa in np.geomspace(10, 1e6, 60):
        for N in range(2, 65):
            assert spdhg.rate(kappa / N, N) < spdhg.rate(kappa, 1)
    # ... and the threshold matters: it fails for a well-conditioned problem
    assert spdhg.rate(0.01 / 2, 2) > spdhg.rate(0.01, 1)


def test_paper_constants_fixture():
    # Section III's printed problems (kappa ~ 70, 20 rigid and 10 non-rigid
    # gates) satisfy Section II-B's condition kappa >= 10, so with Theorem 1's
    # approximations |A_i| ~ |A| and |(A_1..A_N)|^2 ~ N |A|^2 the SPDHG epoch
    # rate l(kappa / N, N) is below PDHG's l(kappa, 1) for both
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        g = json.load(f)
    k = g["kappa"]["value"]
    assert k >= 10
    for N in (g["gates"]["rigid"], g["gates"]["nonrigid"]):
        assert spdhg.rate(k / N, N) < spdhg.rate(k, 1)


def _iteration_matrices(mats, alpha, sigma, tau, theta, p, S_list):
    """Matrices of the homogeneous iteration (d = 0) on the state (x, y, z-bar),
    with z = sum_i A_i^T y_i implied, one per drawn gate set."""
    ops = MatrixOps(mats)
    N = len(mats)
    nx = mats[0].shape[1]
    ny = [m.shape[0] for m in mats]
    dim = nx + sum(ny) + nx
    zero_d = [np.zeros(k) for k in ny]

    def unpack(v):
        x = v[:nx]
        ys, o = [], nx
        for k in ny:
            ys.append(v[o:o + k])
            o += k
        return x, ys, v[o:o + nx]

    out = []
    for S in S_list:
        M = np.zeros((dim, dim))
        for c in range(dim):
            e = np.zeros(dim)
            e[c] = 1
            x, ys, zb = unpack(e)
            st = spdhg.State(x, ys, sum(mats[i].T @ ys[i] for i in range(N)), zb)
            nxt = spdhg.iterate(ops, st, zero_d, alpha, sigma, tau, theta, p, S)
            M[:, c] = np.concatenate([nxt.x] + nxt.y + [nxt.zbar])
        out.append(M)
    return out


@pytest.mark.parametrize("N,alpha,seed", [(1, 0.2, 0), (3, 0.05, 1), (4, 1.0, 2), (8, 0.2, 3)])
def test_pdhg_spectral_radius_within_theorem(N, alpha, seed):
    rng = np.random.default_rng(seed)
    mats = [rng.standard_normal((3, 4)) for _ in range(N)]
    L2 = np.linalg.norm(np.concatenate(mats), 2) ** 2
    sigma, tau, theta, rho = spdhg.step_sizes_pdhg(L2, alpha, N)
    (M,) = _iteration_matrices(mats, alpha, sigma, tau, theta, [1.0] * N, [list(range(N))])
    sr = max(abs(np.linalg.eigvals(M)))
    assert sr ** 2 <= spdhg.rate(L2 / (alpha * N), 1) * (1 + 1e-9)


@pytest.mark.parametrize("N,alpha,seed", [(2, 0.2, 0), (3, 0.05, 1), (5, 1.0, 2), (8, 0.2, 3)])
def test_spdhg_second_moment_within_theorem(N, alpha, seed):
    rng = np.random.default_rng(seed + 10)
    mats = [rng.standard_normal((3, 4)) for _ in range(N)]
    norms = [np.linalg.norm(m, 2) ** 2 for m in mats]
    sigma, tau, theta, rho = spdhg.step_sizes_spdhg(norms, alpha, N)
    Ms = _iteration_matrices(mats, alpha, sigma, tau, theta, [1 / N] * N, [[i] for i in range(N)])
    T = sum(np.kron(M, M) for M in Ms) / N
    sr = max(abs(np.linalg.eigvals(T)))
    kappa = max(norms) / (alpha * N)
    assert sr <= (1 - 2 / (N * (1 + math.sqrt(1 + kappa)))) * (1 + 1e-9)
    assert sr ** N <= spdhg.rate(kappa, N) * (1 + 1e-9)


def _paper_regime(N, kind, seed=0, n=20, na=30, nd=30):
    if kind == "rigid":
        ops = GatedOperators(n, na, nd, "rigid", synth.rigid_params(N, seed + 11, 8.0, 1.5))
    else:
        ops = GatedOperators(n, na, nd, "field", synth.dilatation_fields(n, N, seed + 11) * 0.25)
    x_true = synth.ellipse_phantom(n, seed).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((N, na, nd), seed + 12))
    plain = GatedOperators(n, na, nd, "identity", n_gates=1)
    v0 = synth.random_image(n, 99).astype(np.float64)
    normA, _ = spdhg.gate_norm_sq(plain, 0, v0)
    alpha = normA / 70.0          # kappa = |A|^2 / alpha ~ 70, as in Section III
    return ops, d, alpha, v0


@pytest.mark.parametrize("N,kind", [(4, "rigid"), (5, "field")])
def test_observed_rates_in_paper_regime(N, kind):
    ops, d, alpha, v0 = _paper_regime(N, kind)
    xs, ys = spdhg.saddle_point(ops, d, alpha, dense=True)
    gn = [spdhg.gate_norm_sq(ops, i, v0)[0] for i in range(N)]
    sn, _ = spdhg.stacked_norm_sq(ops, v0)
    k_s, k_p = spdhg.condition_numbers(gn, sn, alpha, N)
    epochs = 24

    sig, tau, th, _ = spdhg.step_sizes_pdhg(sn, alpha, N)
    st = spdhg.State.zeros(ops.n, N, ops.n_angles, ops.n_det)
    dp = []
    for e in range(epochs):
        st = spdhg.pdhg(ops, st, d, alpha, sig, tau, th)
        dp.append(spdhg.dist_sq(st, xs, ys))
    slope_p = np.polyfit(np.arange(6, epochs), np.log(dp[6:]), 1)[0]
    assert slope_p <= math.log(spdhg.rate(k_p, 1)) + 0.02, (slope_p, math.log(spdhg.rate(k_p, 1)))

    sig, tau, th, _ = spdhg.step_sizes_spdhg(gn, alpha, N)
    runs = []
    for seed in range(8):
        st = spdhg.State.zeros(ops.n, N, ops.n_angles, ops.n_det)
        cur = []
        for e in range(epochs):
            st = spdhg.spdhg(ops, st, d, alpha, sig, tau, th, [1 / N] * N, synth.gate_sequence(N, seed, e))
            cur.append(spdhg.dist_sq(st, xs, ys))
        runs.append(cur)
    ds = np.mean(runs, axis=0)
    slope_s = np.polyfit(np.arange(6, epochs), np.log(ds[6:]), 1)[0]
    assert slope_s <= math.log(spdhg.rate(k_s, N)) + 0.05, (slope_s, math.log(spdhg.rate(k_s, N)))
    # Section III: SPDHG is ahead of PDHG after the same number of epochs
    assert ds[-1] < dp[-1]
    # Section II-B: the gate norms stay close to |A|^2 and the stacked norm to N |A|^2
    normA = spdhg.gate_norm_sq(GatedOperators(ops.n, ops.n_angles, ops.n_det, "identity", n_gates=1), 0, v0)[0]
    assert abs(max(gn) / normA - 1) < 0.1 and abs(sn / (N * normA) - 1) < 0.15


def test_gap_nonnegative_and_decreasing():
    ops, d, alpha = small_problem()
    plain = GatedOperators(ops.n, ops.n_angles, ops.n_det, "identity", n_gates=1)
    v0 = synth.random_image(ops.n, 1).astype(np.float64)
    sn, _ = spdhg.stacked_norm_sq(ops, v0)
    sig, tau, th, _ = spdhg.step_sizes_pdhg(sn, alpha, 3)
    st = spdhg.State.zeros(ops.n, 3, ops.n_angles, ops.n_det)
    gaps = []
    for _ in range(40):
        st = spdhg.pdhg(ops, st, d, alpha, sig, tau, th)
        gaps.append(spdhg.duality_gap(ops, st.x, st.y, d, alpha))
    assert min(gaps) >= 0
    assert gaps[-1] < 1e-3 * gaps[0]
    del plain


def test_noise_statistics():
    n, na, nd, N = 32, 40, 46, 4
    ops = GatedOperators(n, na, nd, "rigid", synth.rigid_params(N, 1, 5, 4))
    x = synth.ellipse_phantom(n, 0).astype(np.float64)
    noise = synth.unit_noise((N, na, nd), 2)
    d = spdhg.make_data(ops, x, noise)
    s = 0.01 * np.abs(ops.project(x)).max()
    resid = np.concatenate([(d[i] - ops.A(i, x)).ravel() for i in range(N)])
    assert abs(resid.var() / (s * s / N) - 1) < 0.02
