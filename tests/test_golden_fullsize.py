"""The stored full-size oracle results (tests/golden/fullsize_*.npz) against the
oracle itself, on the CPU: the paper-regime minimisers are recomputed and the
motion-compensated one is closer to the truth (Section III, Figs. 2-3 (c) vs
(d)); the stored data hashes are those of the oracle's data; the stored
metadata match the workloads the GPU tests rebuild."""
import math

import numpy as np
import pytest

import golden_fullsize as gf
import synth
from oracle import projector
from oracle import spdhg as osp
from oracle.operators import GatedOperators


def test_paper_regime_minimisers_recomputed():
    arrays, meta = gf.load("k70")
    for name, pm in meta["problems"].items():
        wl = synth.WORKLOADS[name]
        N = wl.n_gates
        params = wl.rigid() if wl.motion == "rigid" else wl.fields().astype(np.float64)
        M = projector.sparse_matrix(wl.n, wl.n_angles, wl.n_det)
        ops = GatedOperators(wl.n, wl.n_angles, wl.n_det, wl.motion, params, matrix=M)
        plain = GatedOperators(wl.n, wl.n_angles, wl.n_det, "identity", n_gates=N, matrix=M)
        v0 = synth.random_image(wl.n, 17).astype(np.float64)
        norm_a, _ = osp.gate_norm_sq(plain, 0, v0)
        assert math.isclose(norm_a, pm["norm_A_sq"], rel_tol=1e-12)
        alpha = norm_a / wl.kappa
        x_true = wl.image().astype(np.float64)
        d = osp.make_data(ops, x_true, synth.unit_noise((N, wl.n_angles, wl.n_det), wl.noise_seed))
        xs, _ = osp.saddle_point(ops, d, alpha)
        xnm, _ = osp.saddle_point(plain, d, alpha)
        key = pm["key"]
        assert np.linalg.norm(xs - arrays[key + "_xs"]) <= 1e-10 * np.linalg.norm(xs)
        assert np.linalg.norm(xnm - arrays[key + "_xs_nomc"]) <= 1e-10 * np.linalg.norm(xnm)
        err = lambda a: float(np.linalg.norm(a - x_true) / np.linalg.norm(x_true))  # noqa: E731
        assert err(xs) < err(xnm), (name, err(xs), err(xnm))
        # optimality of the stored minimiser: alpha x* + N^-1 sum A_i^*(A_i x* - d_i) = 0
        g = alpha * xs + sum(ops.At(i, ops.A(i, xs) - d[i]) for i in range(N)) / N
        rhs = sum(ops.At(i, d[i]) for i in range(N)) / N
        assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(rhs)


def test_gradient_case_data_hashes():
    # the differentiation case's data are seeded sinograms (no operator): the
    # stored hashes must be theirs
    arrays, meta = gf.load("c5_grad")
    d = 50.0 * np.abs(synth.random_sinograms(16, 720, 730, 13, dtype=np.float64))
    assert [gf.sha(v) for v in d] == [str(v) for v in arrays["d_sha256"]]
    assert meta["gate_sequence"] == [int(g) for g in synth.gate_sequence(16, 11, 0, length=10)]
    sig, tau, th, _ = osp.step_sizes_spdhg([meta["norm_estimate"]] * 16, 1e-3, 16)
    assert meta["sigma"] == sig and meta["tau"] == tau and meta["theta"] == th


@pytest.mark.parametrize("case", ["c2_spdhg", "c2_pdhg", "c3_spdhg"])
def test_fullsize_metadata(case):
    try:
        arrays, meta = gf.load(case)
    except FileNotFoundError:
        pytest.skip(f"{case} not stored")
    wl = synth.WORKLOADS[meta["workload"]]
    assert (meta["n"], meta["n_angles"], meta["n_det"], meta["gates"]) == (wl.n, wl.n_angles, wl.n_det, wl.n_gates)
    N = wl.n_gates
    if meta["algorithm"] == "spdhg":
        sig, tau, th, _ = osp.step_sizes_spdhg([meta["norm_estimate"]] * N, wl.alpha, N)
    else:
        sig, tau, th, _ = osp.step_sizes_pdhg(N * meta["norm_estimate"], wl.alpha, N)
    assert meta["sigma"] == sig and meta["tau"] == tau and meta["theta"] == th
    assert len(arrays["d_sha256"]) == N
    for e in meta["epochs"]:
        assert arrays[f"e{e}_x"].shape == (wl.n, wl.n) and np.all(np.isfinite(arrays[f"e{e}_x"]))
        assert arrays[f"e{e}_y_sample"].shape == arrays["y_index"].shape


def test_rigid_workload_data_hash_of_one_gate():
    # one gate of the 8-rigid-gate workload's data through the plain oracle
    # (projector.forward, no sparse matrix): its float32 bytes hash to the
    # stored value, so the stored iterates were computed on the oracle's data
    try:
        arrays, meta = gf.load("c2_spdhg")
    except FileNotFoundError:
        pytest.skip("c2_spdhg not stored")
    wl = synth.WORKLOADS["ellipses512_rigid8"]
    N = wl.n_gates
    ops = GatedOperators(wl.n, wl.n_angles, wl.n_det, "rigid", wl.rigid())
    x_true = np.asarray(wl.image(), dtype=np.float64)
    scale = 0.01 * float(np.max(np.abs(ops.project(x_true))))
    noise = synth.unit_noise((N, wl.n_angles, wl.n_det), wl.noise_seed)
    i = 5
    d = (ops.A(i, x_true) + (scale / math.sqrt(N)) * noise[i]).astype(np.float32)
    assert gf.sha(d) == str(arrays["d_sha256"][i])
