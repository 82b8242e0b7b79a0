"""Pins of the oracle's SPDHG over gates x angle subsets (the next step named in
the Conclusions): reduction to the gate algorithm for one subset, the row
partition of each gate operator, block norms against a library SVD, the saddle
point as a fixed point, the invariant z = sum_i A_i^* y_i, the step-size
identities, the exact second-moment spectral radius of the block iteration on
tiny problems against the rate bound, and observed rates in the paper's
regime (kappa ~ 70)."""
import math

import numpy as np
import pytest

from oracle import spdhg, subsets
from oracle.operators import GatedOperators
import synth


PARTITIONS = ["contiguous", "paired"]


def small(n=16, na=18, nd=24, N=3, M=3, alpha=5.0, seed=0, partition="contiguous"):
    ops = GatedOperators(n, na, nd, "rigid", synth.rigid_params(N, seed + 1, 6.0, 2.0))
    x_true = synth.ellipse_phantom(n, seed).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((N, na, nd), seed + 2))
    return ops, subsets.BlockOperators(ops, M, partition), d, alpha


def test_subset_bounds():
    assert subsets.subset_bounds(720, 4) == [0, 180, 360, 540, 720]
    assert subsets.subset_bounds(10, 3) == [0, 3, 6, 10]
    assert subsets.subset_bounds(5, 1) == [0, 5]
    with pytest.raises(ValueError):
        subsets.subset_bounds(5, 6)


def test_paired_subsets():
    # every angle with its partner a quarter turn away, each subset two
    # contiguous ranges, all angles exactly once
    parts = subsets.paired_subsets(720, 4)
    assert np.array_equal(parts[0], np.r_[0:90, 360:450])
    assert np.array_equal(parts[3], np.r_[270:360, 630:720])
    assert np.array_equal(np.sort(np.concatenate(parts)), np.arange(720))
    for p in subsets.paired_subsets(18, 3):
        assert set((p + 9) % 18) == set(p)
    with pytest.raises(ValueError):
        subsets.paired_subsets(17, 2)
    ops = GatedOperators(8, 6, 12, "identity", n_gates=1)
    with pytest.raises(ValueError):
        subsets.BlockOperators(ops, 2, [np.array([0, 1, 2]), np.array([2, 3, 4, 5])])


def test_one_subset_is_the_gate_algorithm():
    ops, _, d, alpha = small()
    b1 = subsets.BlockOperators(ops, 1)
    N = ops.n_gates
    sig, tau, th, _ = spdhg.step_sizes_spdhg([3.0e2] * N, alpha, N)
    sig_b, tau_b, th_b, _ = subsets.step_sizes([3.0e2] * N, alpha, N)
    assert sig_b == sig and tau_b == tau and th_b == th
    p = [1.0 / N] * N
    a = spdhg.State.zeros(ops.n, N, ops.n_angles, ops.n_det)
    b = a.copy()
    for k, g in enumerate([2, 0, 0, 1, 2]):
        a = spdhg.iterate(ops, a, d, alpha, sig, tau, th, p, [g])
        b = subsets.iterate(b1, b, d, alpha, sig, tau, th, p, [g])
    for u, v in [(a.x, b.x), (a.z, b.z), (a.zbar, b.zbar)] + list(zip(a.y, b.y)):
        np.testing.assert_allclose(v, u, rtol=0, atol=1e-13 * max(1.0, np.abs(u).max()))


@pytest.mark.parametrize("partition", PARTITIONS)
def test_blocks_partition_each_gate_operator(partition):
    ops, bops, _, _ = small(partition=partition)
    x = synth.random_image(ops.n, 3).astype(np.float64)
    y = synth.random_sinograms(1, ops.n_angles, ops.n_det, 4)[0].astype(np.float64)
    for i in range(ops.n_gates):
        parts = [bops.A(i * bops.n_subsets + s, x) for s in range(bops.n_subsets)]
        np.testing.assert_array_equal(sum(parts), ops.A(i, x))
        for s, part in enumerate(parts):   # zero outside the subset's rows
            keep = np.zeros(ops.n_angles, bool)
            keep[bops.rows(s)] = True
            assert not part[~keep].any()
        np.testing.assert_allclose(sum(bops.At(i * bops.n_subsets + s, y) for s in range(bops.n_subsets)),
                                   ops.At(i, y), rtol=1e-12, atol=1e-12)
    for b in range(bops.n_blocks):   # dot test
        lhs = float(np.vdot(bops.A(b, x), y))
        rhs = float(np.vdot(x, bops.At(b, y)))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("partition", PARTITIONS)
def test_block_norms_against_svd(partition):
    ops, bops, _, _ = small(n=10, na=12, nd=16, N=2, M=3, partition=partition)
    n = ops.n
    v0 = synth.random_image(n, 9).astype(np.float64)
    for i in range(ops.n_gates):
        full = np.zeros((ops.n_angles * ops.n_det, n * n))
        blocks = [np.zeros_like(full) for _ in range(bops.n_subsets)]
        e = np.zeros((n, n))
        for q in range(n * n):
            e[:] = 0
            e.flat[q] = 1
            full[:, q] = ops.A(i, e).ravel()
            for s in range(bops.n_subsets):
                blocks[s][:, q] = bops.A(i * bops.n_subsets + s, e).ravel()
        gate2 = np.linalg.norm(full, 2) ** 2
        b2 = [np.linalg.norm(m, 2) ** 2 for m in blocks]
        for s in range(bops.n_subsets):
            lam, _ = subsets.block_norm_sq(bops, i * bops.n_subsets + s, v0, rtol=1e-14, max_iter=5000)
            assert abs(lam - b2[s]) <= 1e-9 * b2[s]
        # a row partition: max_s |A_b|^2 <= |A_i|^2 <= sum_s |A_b|^2
        assert max(b2) <= gate2 * (1 + 1e-12) and gate2 <= sum(b2) * (1 + 1e-12)


@pytest.mark.parametrize("partition", PARTITIONS)
def test_saddle_point_is_a_fixed_point_of_the_block_iteration(partition):
    ops, bops, d, alpha = small(partition=partition)
    xs, ys = spdhg.saddle_point(ops, d, alpha, dense=True)
    zs = sum(ops.At(i, ys[i]) for i in range(ops.n_gates))
    np.testing.assert_allclose(zs, -2 * alpha * xs, rtol=1e-9, atol=1e-11)
    st = spdhg.State(xs.copy(), [v.copy() for v in ys], zs.copy(), zs.copy())
    nb = bops.n_blocks
    sig, tau, th, _ = subsets.step_sizes([4.0e2] * nb, alpha, ops.n_gates)
    p = [1.0 / nb] * nb
    for b in [0, 4, 8, 3, 7]:
        st = subsets.iterate(bops, st, d, alpha, sig, tau, th, p, [b])
    scale = np.abs(xs).max()
    assert np.abs(st.x - xs).max() <= 1e-9 * scale
    for a, b in zip(st.y, ys):
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("partition", PARTITIONS)
def test_invariant_z_is_sum_of_gate_adjoints(partition):
    ops, bops, d, alpha = small(partition=partition)
    nb = bops.n_blocks
    sig, tau, th, _ = subsets.step_sizes([4.0e2] * nb, alpha, ops.n_gates)
    st = spdhg.State.zeros(ops.n, ops.n_gates, ops.n_angles, ops.n_det)
    st = subsets.spdhg_blocks(bops, st, d, alpha, sig, tau, th, [1.0 / nb] * nb, synth.gate_sequence(nb, 5, 0))
    z = sum(ops.At(i, st.y[i]) for i in range(ops.n_gates))
    np.testing.assert_allclose(st.z, z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_step_size_identities():
    # theta (1 + 2 tau mu_g) = 1 with mu_g = 2 alpha, and tau sigma_b |A_b|^2 <= p / theta,
    # with equality for the largest block
    norms = [3.0, 7.5, 1.2, 7.5, 0.4, 2.2]
    alpha, N = 0.3, 2
    sig, tau, th, rho = subsets.step_sizes(norms, alpha, N)
    p = 1.0 / len(norms)
    assert abs(th * (1 + 4 * alpha * tau) - 1) < 1e-14
    vals = [tau * s * a for s, a in zip(sig, norms)]
    assert max(vals) == pytest.approx(p / th, rel=1e-13)
    assert all(v <= p / th * (1 + 1e-13) for v in vals)
    assert subsets.epoch_rate(norms, alpha, N) == pytest.approx(rho ** len(norms), rel=1e-13)


class _MatrixBlocks:
    """Explicit matrices A_i (rows = data entries) cut into M row subsets."""

    def __init__(self, mats, M, partition="contiguous"):
        self.mats = [np.asarray(m, dtype=np.float64) for m in mats]
        self.n_gates = len(mats)
        self.n_subsets = M
        self.n_blocks = self.n_gates * M
        rows = self.mats[0].shape[0]
        make = {"contiguous": subsets.contiguous_subsets, "paired": subsets.paired_subsets}[partition]
        self.parts = make(rows, M)

    def split(self, b):
        return divmod(int(b), self.n_subsets)

    def rows(self, s):
        return self.parts[s]

    def A(self, b, x):
        i, s = self.split(b)
        out = np.zeros(self.mats[i].shape[0])
        out[self.rows(s)] = (self.mats[i] @ x)[self.rows(s)]
        return out

    def At(self, b, y):
        i, s = self.split(b)
        yy = np.zeros_like(y)
        yy[self.rows(s)] = y[self.rows(s)]
        return self.mats[i].T @ yy


@pytest.mark.parametrize("partition", PARTITIONS)
@pytest.mark.parametrize("N,M,alpha,seed", [(1, 3, 0.2, 0), (2, 2, 0.05, 1), (3, 3, 1.0, 2), (2, 4, 0.2, 3)])
def test_block_second_moment_within_rate(N, M, alpha, seed, partition):
    if partition == "paired" and M > 3:
        pytest.skip("6 data rows pair into at most 3 subsets")
    # exact mean-square contraction of the block iteration (d = 0, error form):
    # T = sum_b p_b M_b (x) M_b; its spectral radius per iteration must not
    # exceed 1 - 2p/(1 + s) of the step-size rule
    rng = np.random.default_rng(seed + 40)
    mats = [rng.standard_normal((6, 4)) for _ in range(N)]
    bops = _MatrixBlocks(mats, M, partition)
    norms = []
    for b in range(bops.n_blocks):
        i, s = bops.split(b)
        norms.append(np.linalg.norm(mats[i][bops.rows(s)], 2) ** 2)
    sig, tau, th, rho = subsets.step_sizes(norms, alpha, N)
    nb = bops.n_blocks
    p = [1.0 / nb] * nb
    nx, ny = 4, 6
    dim = nx + N * ny + nx
    zero_d = [np.zeros(ny) for _ in range(N)]
    Ms = []
    for b in range(nb):
        Mb = np.zeros((dim, dim))
        for c in range(dim):
            e = np.zeros(dim)
            e[c] = 1
            x = e[:nx]
            ys = [e[nx + k * ny: nx + (k + 1) * ny] for k in range(N)]
            zb = e[nx + N * ny:]
            st = spdhg.State(x, [v.copy() for v in ys], sum(mats[i].T @ ys[i] for i in range(N)), zb)
            nxt = subsets.iterate(bops, st, zero_d, alpha, sig, tau, th, p, [b])
            Mb[:, c] = np.concatenate([nxt.x] + nxt.y + [nxt.zbar])
        Ms.append(Mb)
    T = sum(np.kron(m, m) for m in Ms) / nb
    sr = max(abs(np.linalg.eigvals(T)))
    assert sr <= rho * (1 + 1e-9), (sr, rho)
    assert sr ** nb <= subsets.epoch_rate(norms, alpha, N) * (1 + 1e-9)


@pytest.mark.parametrize("partition", PARTITIONS)
def test_observed_rate_in_paper_regime(partition):
    # kappa = |A|^2 / alpha ~ 70 (Section III); 4 rigid gates x 3 angle subsets
    N, M, n, na, nd = 4, 3, 20, 30, 30
    ops = GatedOperators(n, na, nd, "rigid", synth.rigid_params(N, 11, 8.0, 1.5))
    x_true = synth.ellipse_phantom(n, 0).astype(np.float64)
    d = spdhg.make_data(ops, x_true, synth.unit_noise((N, na, nd), 12))
    v0 = synth.random_image(n, 99).astype(np.float64)
    normA, _ = spdhg.gate_norm_sq(GatedOperators(n, na, nd, "identity", n_gates=1), 0, v0)
    alpha = normA / 70.0
    xs, ys = spdhg.saddle_point(ops, d, alpha, dense=True)
    bops = subsets.BlockOperators(ops, M, partition)
    nb = bops.n_blocks
    bn = [subsets.block_norm_sq(bops, b, v0)[0] for b in range(nb)]
    gn = [spdhg.gate_norm_sq(ops, i, v0)[0] for i in range(N)]
    sig, tau, th, _ = subsets.step_sizes(bn, alpha, N)
    r_blocks = subsets.epoch_rate(bn, alpha, N)
    r_gates = spdhg.rate(max(gn) / (alpha * N), N)
    assert r_blocks < r_gates      # the theory's promise for subsets
    epochs = 20
    runs = []
    for seed in range(8):
        st = spdhg.State.zeros(n, N, na, nd)
        cur = []
        for e in range(epochs):
            st = subsets.spdhg_blocks(bops, st, d, alpha, sig, tau, th, [1.0 / nb] * nb,
                                      synth.gate_sequence(nb, seed, e))
            cur.append(spdhg.dist_sq(st, xs, ys))
        runs.append(cur)
    ds = np.mean(runs, axis=0)
    slope = np.polyfit(np.arange(5, epochs), np.log(ds[5:]), 1)[0]
    assert slope <= math.log(r_blocks) + 0.05, (slope, math.log(r_blocks))
