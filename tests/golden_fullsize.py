"""Loads the FP64 oracle's full-size results (tests/golden/fullsize_*.npz,
written by tests/golden/make_fullsize.py from `oracle/` alone) and rebuilds
the data they were computed on."""
from __future__ import annotations

import functools
import hashlib
import json
import math
import os

import numpy as np

import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(case: str):
    """(arrays, meta) of one stored case."""
    z = np.load(os.path.join(HERE, f"fullsize_{case}.npz"))
    arrays = {k: z[k] for k in z.files if k != "meta"}
    return arrays, json.loads(str(z["meta"]))


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float32).tobytes()).hexdigest()


def _data_via_hip(n, na, nd, kind, params, x_true, noise, hashes):
    """float32 data A_i x_true + (s / sqrt(N)) noise_i, s = 0.01 max|A x_true|
    (Section II-A), the ray sums taken from the library's FP64 path
    (bench.hip_data); a gate whose float32 bytes do not hash to the value the
    oracle stored (a value next to a float32 rounding tie) is computed by the
    oracle itself."""
    import bench
    d, differ = bench.hip_data(n, na, nd, kind, params, x_true, noise, hashes)
    if differ:
        from oracle.operators import GatedOperators
        ops = GatedOperators(n, na, nd, kind, np.asarray(params, dtype=np.float64))
        N = len(hashes)
        s_o = 0.01 * float(np.max(np.abs(ops.project(x_true))))
        for i in differ:
            v32 = (ops.A(i, x_true) + (s_o / math.sqrt(N)) * noise[i]).astype(np.float32)
            assert sha(v32) == hashes[i], f"gate {i}: the oracle's data no longer hash to the stored value"
            d[i] = v32
    how = f"FP64 HIP ray sums, hash-checked ({len(differ)} gate(s) recomputed by the oracle)"
    return [v.astype(np.float64) for v in d], how


@functools.lru_cache(maxsize=2)
def workload_data(name: str):
    """float32 data of a 512^2 workload as the oracle made them for the stored
    results. Returns (d list of float64 arrays holding float32 values, how)."""
    wl = synth.WORKLOADS[name]
    hashes = None
    for case in ("c2_spdhg", "c2_pdhg", "c3_spdhg"):
        arrays, meta = load(case)
        if meta["workload"] == name:
            hashes = [str(v) for v in arrays["d_sha256"]]
            break
    assert hashes is not None and len(hashes) == wl.n_gates
    params = wl.rigid() if wl.motion == "rigid" else wl.fields()
    x_true = np.asarray(wl.image(), dtype=np.float64)
    noise = synth.unit_noise((wl.n_gates, wl.n_angles, wl.n_det), wl.noise_seed)
    return _data_via_hip(wl.n, wl.n_angles, wl.n_det, wl.motion, params, x_true, noise, hashes)


def slice_data(sl, n, na, nd, hashes):
    """float32 data of one slice of the batched workload (synth.BatchSlice)."""
    params = sl.rigid() if sl.motion == "rigid" else sl.fields(n)
    x_true = np.asarray(sl.image(n), dtype=np.float64)
    noise = synth.unit_noise((sl.n_gates, na, nd), sl.noise_seed)
    return _data_via_hip(n, na, nd, sl.motion, params, x_true, noise, hashes)
