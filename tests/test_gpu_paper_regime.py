"""Section III on the GPU (FP64, the paper's regime kappa = |A|^2/alpha = 70):
observed per-epoch contraction of PDHG and SPDHG within Theorem 1's rates,
SPDHG ahead of PDHG after the same number of epochs, the norm approximations
of Section II-B, and the motion-compensated minimiser closer to the truth than
the one without motion compensation."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_rates_and_motion_compensation_in_paper_regime():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import bench
    res = bench.paper_experiment()   # 30 epochs, SPDHG averaged over 8 gate sequences
    for name, r in res.items():
        rt = r["rate_per_epoch"]
        assert rt["pdhg_observed"] <= rt["pdhg_theory"] * 1.02, (name, rt)
        assert rt["spdhg_observed_mean"] <= rt["spdhg_theory"] * 1.05, (name, rt)
        assert rt["spdhg_theory"] < rt["pdhg_theory"]
        assert r["dist_sq_spdhg_mean"][-1] < r["dist_sq_pdhg"][-1]
        # Section II-B: max_i |A_i|^2 ~ |A|^2 and |(A_1..A_N)|^2 ~ N |A|^2
        assert abs(r["gate_norm_ratio_max"] - 1) < 0.1 and abs(r["stacked_norm_ratio"] - 1) < 0.15
        e = r["rel_error_vs_truth"]
        assert e["motion_compensated"] < e["no_motion_compensation"]
