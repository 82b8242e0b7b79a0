"""Precision contract: the relative L2 error against the FP64 oracle of every
output of the library, in both precisions, stated and checked against its bar.
Run with -s to see the table; it is also written as JSON to the file that
the environment variable MCR_PRECISION_JSON names, if set."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import Problem, dev, f32, host, need_gpu, rel
import synth
from oracle import projector, spdhg as osp, warp

pytestmark = pytest.mark.gpu

BARS = {"float32": {"op": 1e-5, "epochs": 1e-4}, "float64": {"op": 1e-12, "epochs": 1e-10}}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_precision_table():
    rows = []

    def add(name, dtype, err, bar):
        rows.append({"output": name, "dtype": str(dtype).replace("torch.", ""), "rel_l2": err, "bar": bar})

    n, na, nd = 256, 360, 366
    P = Problem(n, na, nd, 2, "field", phantom="chest", field_scale=1.0)
    R = Problem(n, na, nd, 2, "rigid")
    x = P.x_true
    y = f32(synth.random_sinograms(1, na, nd, 3)[0])
    b = f32(synth.random_image(n, 4))
    ref = {
        "A x": projector.forward(x, na, nd),
        "A^T y": projector.adjoint(y, n),
        "D x (field)": warp.warp(x, *P.ops.pos[1]),
        "D^T b (field)": warp.warp_adjoint(b, *P.ops.pos[1]),
        "D x (rigid)": warp.warp(x, *R.ops.pos[1]),
        "D^T b (rigid)": warp.warp_adjoint(b, *R.ops.pos[1]),
        "A_i x (field)": P.ops.A(1, x),
        "A_i^* y (field)": P.ops.At(1, y),
        "A_i x (rigid)": R.ops.A(1, x),
        "A_i^* y (rigid)": R.ops.At(1, y),
    }
    for dtype in (torch.float32, torch.float64):
        bar = BARS[str(dtype).replace("torch.", "")]["op"]
        hp, hr = P.handle(dtype), R.handle(dtype)
        if dtype == torch.float32:  # the variants the benchmark runs
            hp.autotune(1)
            hr.autotune(1)
        got = {
            "A x": hp.project(dev(x, dtype)), "A^T y": hp.backproject(dev(y, dtype)),
            "D x (field)": hp.warp(1, dev(x, dtype)), "D^T b (field)": hp.warp_adjoint(1, dev(b, dtype)),
            "D x (rigid)": hr.warp(1, dev(x, dtype)), "D^T b (rigid)": hr.warp_adjoint(1, dev(b, dtype)),
            "A_i x (field)": hp.apply_Ai(1, dev(x, dtype)), "A_i^* y (field)": hp.apply_Ai_adjoint(1, dev(y, dtype)),
            "A_i x (rigid)": hr.apply_Ai(1, dev(x, dtype)), "A_i^* y (rigid)": hr.apply_Ai_adjoint(1, dev(y, dtype)),
        }
        for k, v in got.items():
            add(k, dtype, rel(host(v), ref[k]), bar)

    # 50 SPDHG and 50 PDHG epochs (64^2, 4 field gates)
    Q = Problem(64, 96, 92, 4, "field", alpha=1e-3)
    sig, tau, th, _ = osp.step_sizes_spdhg([2.0 * 96 * 64] * 4, Q.alpha, 4)
    p = [0.25] * 4
    refs = osp.State.zeros(64, 4, 96, 92)
    seqs = [synth.gate_sequence(4, 3, e) for e in range(50)]
    for sq in seqs:
        refs = osp.spdhg(Q.ops, refs, Q.d, Q.alpha, sig, tau, th, p, sq)
    psig, ptau, pth, _ = osp.step_sizes_pdhg(4 * 2.0 * 96 * 64, Q.alpha, 4)
    refp = osp.State.zeros(64, 4, 96, 92)
    for _ in range(50):
        refp = osp.pdhg(Q.ops, refp, Q.d, Q.alpha, psig, ptau, pth)
    for dtype in (torch.float32, torch.float64):
        bar = BARS[str(dtype).replace("torch.", "")]["epochs"]
        h = Q.handle(dtype)
        if dtype == torch.float32:
            h.autotune(1)
        d = [dev(v, dtype) for v in Q.d]
        st = h.zero_state()
        for sq in seqs:
            h.spdhg_epoch(st, d, Q.alpha, sig, tau, th, p, sq)
        yg = np.concatenate([host(v).ravel() for v in st.y])
        add("SPDHG x after 50 epochs", dtype, rel(host(st.x), refs.x), bar)
        add("SPDHG y after 50 epochs", dtype, rel(yg, np.concatenate([v.ravel() for v in refs.y])), bar)
        add("SPDHG z-bar after 50 epochs", dtype, rel(host(st.zbar), refs.zbar), bar)
        st = h.zero_state()
        for _ in range(50):
            h.pdhg_epoch(st, d, Q.alpha, psig, ptau, pth)
        add("PDHG x after 50 epochs", dtype, rel(host(st.x), refp.x), bar)
        # FP64 diagnostics on the device (whatever the handle's dtype)
        v0 = f32(synth.random_image(64, 9))
        lam, _ = h.power_norm_sq(2, dev(v0, torch.float64), max_iter=300, rtol=1e-13)
        lam_o, _ = osp.gate_norm_sq(Q.ops, 2, v0, rtol=1e-13, max_iter=300)
        add("|A_i|^2 (FP64 power iteration)", dtype, abs(lam - lam_o) / lam_o, 1e-10)
        xs = f32(refs.x)
        dd = [dev(v, dtype) for v in Q.d]
        obj = h.objective(dev(xs, dtype), dd, Q.alpha)
        add("objective O(x) (FP64)", dtype, abs(obj - osp.objective(Q.ops, xs, Q.d, Q.alpha)) /
            abs(osp.objective(Q.ops, xs, Q.d, Q.alpha)), 1e-12)

    width = max(len(r["output"]) for r in rows)
    print()
    for r in rows:
        print(f"{r['output']:{width}s}  {r['dtype']:8s}  {r['rel_l2']:.2e}  (bar {r['bar']:.0e})")
    out = os.environ.get("MCR_PRECISION_JSON")
    if out:
        with open(out, "w") as f:
            json.dump(rows, f, indent=1)
    for r in rows:
        assert r["rel_l2"] <= r["bar"], r
