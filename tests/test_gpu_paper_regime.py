"""Section III on the GPU (FP64, the paper's regime kappa = |A|^2/alpha = 70):
observed per-epoch contraction of PDHG and SPDHG within Theorem 1's rates,
SPDHG ahead of PDHG after the same number of epochs, the norm approximations
of Section II-B, and the motion-compensated minimiser closer to the truth than
the one without motion compensation. The distances are measured to the FP64
oracle's saddle point (stored by tests/golden/make_fullsize.py, case k70) on
the oracle's data, and the library's conjugate-gradient minimisers are
checked against the oracle's."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _reference():
    """alpha, data and minimisers of both problems from the oracle: alpha and
    x* (with and without motion compensation) as stored, the data and
    y_i* = (2/N)(A_i x* - d_i) recomputed by the oracle (128^2: fast)."""
    import golden_fullsize as gf
    from oracle import spdhg as osp
    from oracle.operators import GatedOperators
    arrays, meta = gf.load("k70")
    out = {}
    for name, pm in meta["problems"].items():
        wl = synth.WORKLOADS[name]
        N = wl.n_gates
        params = wl.rigid() if wl.motion == "rigid" else wl.fields().astype(np.float64)
        ops = GatedOperators(wl.n, wl.n_angles, wl.n_det, wl.motion, params)
        d = osp.make_data(ops, wl.image().astype(np.float64), synth.unit_noise((N, wl.n_angles, wl.n_det),
                                                                               wl.noise_seed))
        xs = arrays[pm["key"] + "_xs"]
        ys = [(2.0 / N) * (ops.A(i, xs) - d[i]) for i in range(N)]
        out[name] = {"alpha": pm["alpha"], "d": d, "xs": xs, "ys": ys, "xs_nomc": arrays[pm["key"] + "_xs_nomc"],
                     "norm_A_sq": pm["norm_A_sq"], "stacked_norm_sq": pm["stacked_norm_sq"],
                     "gate_norms": arrays[pm["key"] + "_gate_norms"]}
    return out


def test_rates_and_motion_compensation_in_paper_regime():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import bench
    ref = _reference()
    res = bench.paper_experiment(reference=ref)   # 30 epochs, SPDHG averaged over 8 gate sequences
    for name, r in res.items():
        rt = r["rate_per_epoch"]
        assert rt["pdhg_observed"] <= rt["pdhg_theory"] * 1.02, (name, rt)
        assert rt["spdhg_observed_mean"] <= rt["spdhg_theory"] * 1.05, (name, rt)
        assert rt["spdhg_theory"] < rt["pdhg_theory"]
        assert r["dist_sq_spdhg_mean"][-1] < r["dist_sq_pdhg"][-1]
        # both decrease towards the oracle's saddle point by orders of magnitude
        assert r["dist_sq_spdhg_mean"][-1] < 1e-2 * r["dist_sq_spdhg_mean"][0]
        # Section II-B: max_i |A_i|^2 ~ |A|^2 and |(A_1..A_N)|^2 ~ N |A|^2
        assert abs(r["gate_norm_ratio_max"] - 1) < 0.1 and abs(r["stacked_norm_ratio"] - 1) < 0.15
        # the library's FP64 norms agree with the oracle's power iterations
        rf = ref[name]
        assert math.isclose(r["norm_A_sq"], rf["norm_A_sq"], rel_tol=1e-9)
        assert math.isclose(r["kappa_pdhg"] * rf["alpha"] * r["gates"], rf["stacked_norm_sq"], rel_tol=1e-9)
        # the library's conjugate-gradient minimisers are the oracle's
        vo = r["oracle_minimisers"]
        assert vo["xs_cg_rel"] < 1e-9 and vo["xs_nomc_cg_rel"] < 1e-9, vo
        # motion compensation helps: on the oracle's minimisers
        e = vo["rel_error_vs_truth"]
        assert e["motion_compensated"] < e["no_motion_compensation"], e
