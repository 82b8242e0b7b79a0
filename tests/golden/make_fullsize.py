"""Writes the FP64 oracle's results at the full workload sizes (tests/golden/fullsize_*.npz).

Every number stored here comes from `oracle/` (and the seeded inputs of
`synth/`); nothing is read from the HIP library. The GPU tests compare the
library's float32 and FP64 runs of the same problems against these files.

Cases (run one per process; they are independent):

  c2_spdhg  512^2 ellipse phantom, 720 angles x 730 bins, 8 rigid gates
            (rotation +-8 deg, shift +-10 px), alpha = 1e-3: 50 SPDHG epochs
            (Algorithm 1, serial uniform sampling, gate draws (3, epoch)).
  c2_pdhg   the same problem, 50 PDHG epochs (every gate every iteration).
  c3_spdhg  512^2 chest-like phantom, 720 x 730, 16 displacement-field gates,
            alpha = 1e-3: 100 SPDHG epochs, the state kept after 50 and 100.
  c5_grad   512^2 ellipse phantom, 720 x 730, 16 rigid gates: loss
            |x^10 - x_true|^2 after 10 unrolled SPDHG iterations from
            0.8 x_true and its gradient with respect to the starting image and
            the 48 rigid motion parameters (transposed iteration map).
  c4_batch  four slices of the batched workload (synth.batched_slices:
            256^2, 360 x 366; slices 5, 7, 10, 14 with 32, 6, 12 and 20
            gates, field and rigid motion), alpha = 1e-3 each: 5 SPDHG epochs
            per slice (gate draws (500 + slice, epoch)); x and z-bar in full
            after the last epoch, at 4096 seeded pixels after the others; 256
            sampled dual entries per gate.
  k70       the paper's regime (Section III: kappa = |A|^2 / alpha = 70) at
            128^2, 120 x 182: for 20 rigid gates on the ellipse phantom and 10
            dilatation gates on the chest phantom, |A|^2, |A_i|^2 and the
            stacked norm by power iteration, alpha, and the saddle point x*
            with and without motion compensation (D_i = I, same data).

Data: d_i = A_i x_true + noise with per-entry variance s^2 / N,
s = 0.01 max|A x_true| (Section II-A), rounded to float32 (the form both sides
consume); the SHA-256 of each gate's float32 bytes is stored so that a test
can show that its data are these. Step sizes are the oracle's rule
(Theorem 1) evaluated at the fixed norm estimate 3.7e5 for every gate: step
sizes are explicit inputs of both sides, so any positive values do.

At 512^2 the projector is applied as the oracle's sparse matrix (the same
weights as `projector.forward`, summed per ray; pinned equal to it), which
takes about 1.3 s per SPDHG iteration on one core instead of 15 s.

    python tests/golden/make_fullsize.py c2_spdhg   # ~12 min, ~9 GB RAM
    python tests/golden/make_fullsize.py c2_pdhg    # ~12 min
    python tests/golden/make_fullsize.py c3_spdhg   # ~40 min
    python tests/golden/make_fullsize.py c5_grad    # ~3 min
    python tests/golden/make_fullsize.py c4_batch   # ~3 min
    python tests/golden/make_fullsize.py k70        # ~2 min
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import grad as ograd  # noqa: E402
from oracle import projector  # noqa: E402
from oracle import spdhg as osp  # noqa: E402
from oracle.operators import GatedOperators  # noqa: E402

NORM_ESTIMATE = 3.7e5          # |A_i|^2 used for the step sizes of the 512^2 cases
Y_SAMPLES = 4096               # sampled dual entries per gate
SAMPLE_SEED = 0x5A3           # seed of the sampled dual entries


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def sha(a32) -> str:
    return hashlib.sha256(np.ascontiguousarray(a32, dtype=np.float32).tobytes()).hexdigest()


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def problem_512(name: str, matrix):
    """The oracle's gated operators, x_true and float32 data of a 512^2 workload."""
    wl = synth.WORKLOADS[name]
    if wl.motion == "rigid":
        params = wl.rigid()
    else:
        params = wl.fields().astype(np.float64)
    ops = GatedOperators(wl.n, wl.n_angles, wl.n_det, wl.motion, params, matrix=matrix)
    x_true = f32(wl.image())
    noise = synth.unit_noise((wl.n_gates, wl.n_angles, wl.n_det), wl.noise_seed)
    d = [f32(v) for v in osp.make_data(ops, x_true, noise)]
    return wl, ops, x_true, d


def y_sample(N, na, nd, count=Y_SAMPLES):
    g = np.random.Generator(np.random.PCG64([SAMPLE_SEED, N, na, nd]))
    return g.integers(0, na * nd, size=(N, count)).astype(np.int64)


def state_arrays(st, prefix, idx, pix=None):
    """x and z-bar in full (pix None) or at the pixels `pix`, the sampled
    duals, and the norms of every y_i and of z."""
    N = len(st.y)
    out = {
        f"{prefix}z_norm": np.array(float(np.linalg.norm(st.z))),
        f"{prefix}y_norm": np.array([float(np.linalg.norm(v)) for v in st.y]),
        f"{prefix}y_sample": np.stack([st.y[i].ravel()[idx[i]] for i in range(N)]),
    }
    if pix is None:
        out[f"{prefix}x"] = st.x
        out[f"{prefix}zbar"] = st.zbar
    else:
        out[f"{prefix}x_sample"] = st.x.ravel()[pix]
        out[f"{prefix}zbar_sample"] = st.zbar.ravel()[pix]
    return out


def save(case, arrays, meta):
    path = os.path.join(HERE, f"fullsize_{case}.npz")
    arrays = dict(arrays)
    arrays["meta"] = np.array(json.dumps(meta, sort_keys=True))
    np.savez_compressed(path, **arrays)
    log(f"wrote {path}")


def common_meta(wl, case, sig, tau, th, p):
    return {
        "case": case, "workload": wl.name, "n": wl.n, "n_angles": wl.n_angles, "n_det": wl.n_det,
        "gates": wl.n_gates, "motion": wl.motion, "alpha": wl.alpha, "phantom": wl.phantom,
        "seeds": {"phantom": wl.phantom_seed, "motion": wl.motion_seed, "noise": wl.noise_seed,
                  "gates": wl.gate_seed, "y_sample": SAMPLE_SEED},
        "norm_estimate": NORM_ESTIMATE, "sigma": list(sig), "tau": tau, "theta": th, "p": list(p),
        "writer": "tests/golden/make_fullsize.py (oracle only)",
    }


def run_spdhg(case, name, snapshots):
    t0 = time.time()
    M = projector.sparse_matrix(512, 720, 730)
    log(f"{case}: matrix assembled in {time.time() - t0:.0f} s ({M.nnz} weights)")
    wl, ops, x_true, d = problem_512(name, M)
    N = wl.n_gates
    sig, tau, th, _ = osp.step_sizes_spdhg([NORM_ESTIMATE] * N, wl.alpha, N)
    p = [1.0 / N] * N
    idx = y_sample(N, wl.n_angles, wl.n_det)
    st = osp.State.zeros(wl.n, N, wl.n_angles, wl.n_det)
    arrays = {"d_sha256": np.array([sha(v) for v in d]), "y_index": idx}
    for e in range(max(snapshots)):
        st = osp.spdhg(ops, st, d, wl.alpha, sig, tau, th, p, synth.gate_sequence(N, wl.gate_seed, e))
        if (e + 1) % 5 == 0:
            log(f"{case}: epoch {e + 1} ({time.time() - t0:.0f} s)")
        if e + 1 in snapshots:
            arrays.update(state_arrays(st, f"e{e + 1}_", idx))
    meta = common_meta(wl, case, sig, tau, th, p)
    meta.update({"algorithm": "spdhg", "epochs": list(snapshots), "gate_sequence": "synth.gate_sequence(N, 3, epoch)"})
    save(case, arrays, meta)


def run_pdhg(case, name, epochs):
    t0 = time.time()
    M = projector.sparse_matrix(512, 720, 730)
    log(f"{case}: matrix assembled in {time.time() - t0:.0f} s")
    wl, ops, x_true, d = problem_512(name, M)
    N = wl.n_gates
    sig, tau, th, _ = osp.step_sizes_pdhg(N * NORM_ESTIMATE, wl.alpha, N)
    idx = y_sample(N, wl.n_angles, wl.n_det)
    st = osp.State.zeros(wl.n, N, wl.n_angles, wl.n_det)
    for e in range(epochs):
        st = osp.pdhg(ops, st, d, wl.alpha, sig, tau, th, iters=1)
        if (e + 1) % 5 == 0:
            log(f"{case}: epoch {e + 1} ({time.time() - t0:.0f} s)")
    arrays = {"d_sha256": np.array([sha(v) for v in d]), "y_index": idx}
    arrays.update(state_arrays(st, f"e{epochs}_", idx))
    meta = common_meta(wl, case, sig, tau, th, [1.0] * N)
    meta.update({"algorithm": "pdhg", "epochs": [epochs]})
    save(case, arrays, meta)


def run_grad(case):
    """10 unrolled SPDHG iterations at 512^2 with 16 rigid gates; the data are
    seeded synthetic sinograms of the size of the phantom's line integrals
    (50 |standard normal|), which is all the identities being tested need."""
    t0 = time.time()
    M = projector.sparse_matrix(512, 720, 730)
    log(f"{case}: matrix assembled in {time.time() - t0:.0f} s")
    n, na, nd, N, alpha = 512, 720, 730, 16, 1e-3
    params = synth.rigid_params(N, 1, 8.0, 10.0)
    ops = GatedOperators(n, na, nd, "rigid", params, matrix=M)
    x_true = f32(synth.ellipse_phantom(n, 0))
    d = [f32(v) for v in 50.0 * np.abs(synth.random_sinograms(N, na, nd, 13, dtype=np.float64))]
    sig, tau, th, _ = osp.step_sizes_spdhg([NORM_ESTIMATE] * N, alpha, N)
    p = [1.0 / N] * N
    seq = [int(g) for g in synth.gate_sequence(N, 11, 0, length=10)]
    x0 = f32(0.8 * x_true)
    loss, gx, gm = ograd.unrolled_loss_and_grad(ops, x0, d, alpha, sig, tau, th, p, seq, x_true)
    log(f"{case}: loss {loss:.6e} in {time.time() - t0:.0f} s")
    meta = {"case": case, "n": n, "n_angles": na, "n_det": nd, "gates": N, "alpha": alpha,
            "motion": "rigid: synth.rigid_params(16, 1, 8, 10)", "phantom": "ellipses seed 0",
            "x0": "float32(0.8 x_true)", "target": "x_true",
            "data": "float32(50 |synth.random_sinograms(16, 720, 730, 13)|)",
            "gate_sequence": seq, "sigma": list(sig), "tau": tau, "theta": th, "p": p,
            "norm_estimate": NORM_ESTIMATE, "writer": "tests/golden/make_fullsize.py (oracle only)"}
    save(case, {"loss": np.array(loss), "grad_x0": gx, "grad_motion": gm,
                 "d_sha256": np.array([sha(v) for v in d])}, meta)


C4_SLICES = (5, 7, 10, 14)


def run_batch(case, epochs=5):
    """Slices of the batched workload, each its own problem (Section II-A
    model per slice), 5 SPDHG epochs; step sizes from the norm estimate
    2 n_angles n (any positive values are valid inputs)."""
    t0 = time.time()
    n, na, nd, alpha = 256, 360, 366, 1e-3
    M = projector.sparse_matrix(n, na, nd)
    slices = [sl for sl in synth.batched_slices() if sl.index in C4_SLICES]
    arrays, meta = {}, {"case": case, "n": n, "n_angles": na, "n_det": nd, "alpha": alpha, "epochs": epochs,
                        "slices": [], "writer": "tests/golden/make_fullsize.py (oracle only)"}
    for sl in slices:
        N = sl.n_gates
        params = sl.rigid() if sl.motion == "rigid" else sl.fields(n).astype(np.float64)
        ops = GatedOperators(n, na, nd, sl.motion, params, matrix=M)
        x_true = f32(sl.image(n))
        noise = synth.unit_noise((N, na, nd), sl.noise_seed)
        d = [f32(v) for v in osp.make_data(ops, x_true, noise)]
        sig, tau, th, _ = osp.step_sizes_spdhg([2.0 * na * n] * N, alpha, N)
        p = [1.0 / N] * N
        idx = y_sample(N, na, nd, count=256)  # 256 dual entries per gate (70 gates, 5 epochs)
        pix = np.random.Generator(np.random.PCG64([SAMPLE_SEED, sl.index, n])).integers(0, n * n, size=Y_SAMPLES)
        st = osp.State.zeros(n, N, na, nd)
        key = f"s{sl.index}_"
        arrays[key + "d_sha256"] = np.array([sha(v) for v in d])
        arrays[key + "y_index"] = idx
        arrays[key + "pixel_index"] = pix
        for e in range(epochs):
            st = osp.spdhg(ops, st, d, alpha, sig, tau, th, p, synth.gate_sequence(N, sl.gate_seed, e))
            arrays.update(state_arrays(st, f"{key}e{e + 1}_", idx, None if e + 1 == epochs else pix))
        meta["slices"].append({"index": sl.index, "gates": N, "motion": sl.motion, "sigma": sig, "tau": tau,
                               "theta": th, "p": p, "gate_seed": sl.gate_seed})
        log(f"{case}: slice {sl.index} ({N} {sl.motion} gates) done ({time.time() - t0:.0f} s)")
    save(case, arrays, meta)


def run_k70(case):
    """Section III's regime at 128^2: norms, alpha = |A|^2 / 70 and the
    minimisers with and without motion compensation."""
    arrays = {}
    meta = {"case": case, "writer": "tests/golden/make_fullsize.py (oracle only)", "problems": {}}
    for name in ("ellipses128_rigid20_k70", "chest128_field10_k70"):
        t0 = time.time()
        wl = synth.WORKLOADS[name]
        n, na, nd, N = wl.n, wl.n_angles, wl.n_det, wl.n_gates
        params = wl.rigid() if wl.motion == "rigid" else wl.fields().astype(np.float64)
        M = projector.sparse_matrix(n, na, nd)
        ops = GatedOperators(n, na, nd, wl.motion, params, matrix=M)
        plain = GatedOperators(n, na, nd, "identity", n_gates=N, matrix=M)
        v0 = synth.random_image(n, 17).astype(np.float64)
        norm_a, _ = osp.gate_norm_sq(plain, 0, v0)
        alpha = norm_a / wl.kappa
        gn = [osp.gate_norm_sq(ops, i, v0)[0] for i in range(N)]
        sn, _ = osp.stacked_norm_sq(ops, v0)
        x_true = wl.image().astype(np.float64)
        noise = synth.unit_noise((N, na, nd), wl.noise_seed)
        d = osp.make_data(ops, x_true, noise)
        xs, _ = osp.saddle_point(ops, d, alpha)
        xnm, _ = osp.saddle_point(plain, d, alpha)
        key = name.split("_")[1]
        arrays[f"{key}_xs"] = xs
        arrays[f"{key}_xs_nomc"] = xnm
        arrays[f"{key}_gate_norms"] = np.array(gn)
        err = lambda a: float(np.linalg.norm(a - x_true) / np.linalg.norm(x_true))  # noqa: E731
        meta["problems"][name] = {
            "key": key, "n": n, "n_angles": na, "n_det": nd, "gates": N, "motion": wl.motion,
            "kappa": wl.kappa, "norm_A_sq": norm_a, "alpha": alpha, "stacked_norm_sq": sn,
            "data": "float64, not rounded (the paper-regime runs are FP64)",
            "rel_error_vs_truth": {"motion_compensated": err(xs), "no_motion_compensation": err(xnm)},
            "power_iteration": "v0 = synth.random_image(n, 17), rtol 1e-12, at most 500 iterations",
            "saddle_point": "conjugate gradients to a relative residual of 1e-13"}
        log(f"{case}: {name} done in {time.time() - t0:.0f} s: {meta['problems'][name]['rel_error_vs_truth']}")
    save(case, arrays, meta)


CASES = {
    "c2_spdhg": lambda: run_spdhg("c2_spdhg", "ellipses512_rigid8", (50,)),
    "c2_pdhg": lambda: run_pdhg("c2_pdhg", "ellipses512_rigid8", 50),
    "c3_spdhg": lambda: run_spdhg("c3_spdhg", "chest512_field16", (50, 100)),
    "c5_grad": lambda: run_grad("c5_grad"),
    "c4_batch": lambda: run_batch("c4_batch"),
    "k70": lambda: run_k70("k70"),
}


if __name__ == "__main__":
    todo = sys.argv[1:] or list(CASES)
    for c in todo:
        if c not in CASES:
            raise SystemExit(f"unknown case {c}; choose from {sorted(CASES)}")
    for c in todo:
        CASES[c]()
