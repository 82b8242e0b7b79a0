"""Writes tests/golden/paper_constants.json.

The problem constants are the paper's (each entry cites where); nothing in
the file is computed. Run from the repository root:
python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


def main():
    kappa = 70.0
    data = {
        "image_size": {"value": [100, 100], "cite": "Section III, Description"},
        "sinogram_size": {"value": [200, 200], "angles": 200, "geometry": "2D parallel beam",
                          "cite": "Section III, Description"},
        "gates": {"rigid": 20, "nonrigid": 10, "cite": "Section III, Description"},
        "kappa": {"value": kappa, "approx": True, "cite": "Section III, Description (both models)"},
        "norm_approximations": {"max_gate_vs_A": 0.03, "stacked_vs_N_A": 0.08,
                                "cite": "Section II-B, after Theorem 1"},
        "comparison_epoch": {"value": 30, "cite": "Section III, Results; Figs. 2 and 3 (e), (f)"},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_constants.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
