"""GPU tests of the batched SPDHG epoch: equal, bit for bit, to running each
slice through its own handle with the same gate draws; graph replays equal to
plain launches over several epochs; one batch against the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_common import F32_EPOCHS, F32_OP, Problem, dev, f32, host, need_gpu, rel, rel_max
import synth
from oracle import spdhg as osp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _make(n, na, nd, ngs, seed=0, field_every=2):
    """Slices with mixed motion: every field_every-th slice non-rigid."""
    probs = []
    for s, ng in enumerate(ngs):
        kind = "field" if s % field_every == 1 else "rigid"
        probs.append(Problem(n, na, nd, ng, kind, alpha=1e-2, seed=seed + 17 * s))
    return probs


def _batch(probs, dtype=torch.float32):
    from paper_2410_10503_amd import BatchHandle
    P0 = probs[0]
    motion = [m for P in probs for m in P.motion()]
    return BatchHandle(P0.n, P0.na, P0.nd, [P.N for P in probs], motion, dtype=dtype)


def _params(probs):
    alpha = [P.alpha for P in probs]
    sig, tau, th, p = [], [], [], []
    for P in probs:
        s_, t_, th_, _ = osp.step_sizes_spdhg([2.0 * P.na * P.n] * P.N, P.alpha, P.N)
        sig += s_
        p += [1.0 / P.N] * P.N
        tau.append(t_)
        th.append(th_)
    return alpha, sig, tau, th, p


def _seqs(probs, epoch):
    return [list(synth.gate_sequence(P.N, 40 + i, epoch)) for i, P in enumerate(probs)]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_per_slice(use_graph):
    probs = _make(64, 48, 92, [2, 5, 3, 7, 1, 4])
    bh = _batch(probs)
    bh.set_variant(2, 4, 4)
    alpha, sig, tau, th, p = _params(probs)
    st = bh.zero_batch_state()
    d = torch.cat([torch.stack([dev(v, torch.float32) for v in P.d]) for P in probs]).contiguous()
    singles = []
    for P in probs:
        h = P.handle(torch.float32)
        h.set_variant(2, 4, 4)
        singles.append((h, h.zero_state(), [dev(v, torch.float32) for v in P.d]))
    for e in range(3):
        seqs = _seqs(probs, e)
        bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, [g for sq in seqs for g in sq], use_graph=use_graph)
        for i, (P, (h, s1, d1)) in enumerate(zip(probs, singles)):
            o = bh.offsets[i]
            h.spdhg_epoch(s1, d1, alpha[i], sig[o:o + P.N], tau[i], th[i], p[o:o + P.N], seqs[i])
    torch.cuda.synchronize()
    for i, (P, (h, s1, d1)) in enumerate(zip(probs, singles)):
        o = bh.offsets[i]
        assert torch.equal(st["x"][i], s1.x)
        assert torch.equal(st["z"][i], s1.z)
        assert torch.equal(st["zbar"][i], s1.zbar)
        for k in range(P.N):
            assert torch.equal(st["y"][o + k], s1.y[k])


def test_graph_replays_equal_plain_launches():
    probs = _make(48, 40, 70, [3, 6, 2, 4])
    alpha, sig, tau, th, p = _params(probs)
    d = torch.cat([torch.stack([dev(v, torch.float32) for v in P.d]) for P in probs]).contiguous()
    a, b = _batch(probs), _batch(probs)
    sa, sb = a.zero_batch_state(), b.zero_batch_state()
    for e in range(5):
        seq = [g for sq in _seqs(probs, e) for g in sq]
        a.batch_spdhg_epoch(sa, d, alpha, sig, tau, th, p, seq, use_graph=True)
        b.batch_spdhg_epoch(sb, d, alpha, sig, tau, th, p, seq, use_graph=False)
        torch.cuda.synchronize()
        _ = float(sa["x"].abs().sum())  # eager work between replays
        for k in ("x", "z", "zbar", "y"):
            assert torch.equal(sa[k], sb[k]), (e, k)


def test_batch_against_oracle():
    probs = _make(40, 36, 60, [3, 2, 4])
    bh = _batch(probs)
    alpha, sig, tau, th, p = _params(probs)
    d = torch.cat([torch.stack([dev(v, torch.float32) for v in P.d]) for P in probs]).contiguous()
    st = bh.zero_batch_state()
    refs = [osp.State.zeros(P.n, P.N, P.na, P.nd) for P in probs]
    for e in range(2):
        seqs = _seqs(probs, e)
        bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, [g for sq in seqs for g in sq])
        for i, P in enumerate(probs):
            o = bh.offsets[i]
            refs[i] = osp.spdhg(P.ops, refs[i], P.d, alpha[i], sig[o:o + P.N], tau[i], th[i], p[o:o + P.N], seqs[i])
    for i, P in enumerate(probs):
        assert rel(host(st["x"][i]), refs[i].x) < F32_OP * 10
        assert rel(host(st["zbar"][i]), refs[i].zbar) < F32_OP * 10


@pytest.mark.parametrize("dtype,bar", [(torch.float32, F32_EPOCHS), (torch.float64, 1e-10)])
def test_batch_slices_against_oracle_five_epochs(dtype, bar):
    # four slices of the batched workload (256^2, 360 x 366; 32, 6, 12 and 20
    # gates, field and rigid) in one batch handle, 5 epochs, after each epoch
    # x, z-bar and sampled duals of every slice against the FP64 oracle's
    # stored iterates (tests/golden/make_fullsize.py, case c4_batch)
    import golden_fullsize as gf
    from paper_2410_10503_amd import BatchHandle
    arrays, meta = gf.load("c4_batch")
    n, na, nd, alpha = meta["n"], meta["n_angles"], meta["n_det"], meta["alpha"]
    want = [m["index"] for m in meta["slices"]]
    slices = sorted((sl for sl in synth.batched_slices() if sl.index in want), key=lambda sl: want.index(sl.index))
    motion, d_all, ngs = [], [], []
    for sl in slices:
        if sl.motion == "rigid":
            motion += [("rigid", tuple(float(v) for v in r)) for r in sl.rigid()]
        else:
            f = torch.from_numpy(sl.fields(n)).cuda()
            motion += [("field", f[i].contiguous()) for i in range(sl.n_gates)]
        dd, how = gf.slice_data(sl, n, na, nd, [str(v) for v in arrays[f"s{sl.index}_d_sha256"]])
        print(f"slice {sl.index}: data {how}", flush=True)
        d_all += dd
        ngs.append(sl.n_gates)
    bh = BatchHandle(n, na, nd, ngs, motion, dtype=dtype)
    if dtype == torch.float32:
        bh.autotune(max(1, round(sum(ngs) / max(ngs))))
    d = torch.stack([dev(v, dtype) for v in d_all]).contiguous()
    sig, tau, th, p = [], [], [], []
    for m in meta["slices"]:
        sig += m["sigma"]
        p += m["p"]
        tau.append(m["tau"])
        th.append(m["theta"])
    st = bh.zero_batch_state()
    for e in range(meta["epochs"]):
        seq = [int(g) for sl in slices for g in synth.gate_sequence(sl.n_gates, sl.gate_seed, e)]
        bh.batch_spdhg_epoch(st, d, [alpha] * len(slices), sig, tau, th, p, seq, use_graph=True)
        torch.cuda.synchronize()
        for i, sl in enumerate(slices):
            key = f"s{sl.index}_e{e + 1}_"
            o = bh.offsets[i]
            idx = arrays[f"s{sl.index}_y_index"]
            pix = arrays[f"s{sl.index}_pixel_index"]
            ys = np.stack([host(st["y"][o + k]).ravel()[idx[k]] for k in range(sl.n_gates)])
            xs, zs = host(st["x"][i]), host(st["zbar"][i])
            if key + "x" in arrays:      # in full after the last epoch, sampled pixels before
                pairs = (("x", xs), ("zbar", zs))
            else:
                pairs = (("x_sample", xs.ravel()[pix]), ("zbar_sample", zs.ravel()[pix]))
            for name, got in pairs + (("y_sample", ys),):
                ref = arrays[key + name]
                a, b = rel(got, ref), rel_max(got, ref)
                assert a < bar and b < bar, (dtype, e, sl.index, name, a, b)
    print(f"{dtype}: batch of slices {want} within {bar:g} of the oracle after each of {meta['epochs']} epochs",
          flush=True)


def test_batched_workload_shape():
    # 64 slices of 256^2, 360 x 366, gate counts uniform in {4..32}, mixed
    # motion: one graph-replayed epoch equals the per-slice form on sampled slices
    rng = np.random.default_rng(4)
    ngs = [int(v) for v in rng.integers(4, 33, size=64)]
    probs = _make(256, 360, 366, ngs)
    bh = _batch(probs)
    alpha, sig, tau, th, p = _params(probs)
    # data: synthetic sinograms of the right magnitude (no operator needed here)
    d = (torch.from_numpy(synth.random_sinograms(sum(ngs), 360, 366, 5)).to("cuda").abs() * 50.0).contiguous()
    variant = bh.autotune(1)
    st = bh.zero_batch_state()
    seqs = _seqs(probs, 0)
    bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, [g for sq in seqs for g in sq], use_graph=True)
    torch.cuda.synchronize()
    for i in (0, 17, 40, 63):
        P = probs[i]
        h = P.handle(torch.float32)
        h.set_variant(variant["fwd"], variant["adj_px"], variant["adj_shares"])
        o = bh.offsets[i]
        s1 = h.zero_state()
        h.spdhg_epoch(s1, [d[o + k] for k in range(P.N)], alpha[i], sig[o:o + P.N], tau[i], th[i], p[o:o + P.N],
                      seqs[i])
        assert rel(host(st["x"][i]), host(s1.x)) < 1e-6


def test_graph_follows_motion_and_variant_changes():
    # a captured epoch bakes in the projector variants and the transposed
    # warp's window radius: after set_motion (a compressing field that needs a
    # wider window) and after set_variant, graph replays still equal plain
    # launches on a twin handle
    probs = _make(48, 40, 70, [3, 4, 2], field_every=2)
    alpha, sig, tau, th, p = _params(probs)
    d = torch.cat([torch.stack([dev(v, torch.float32) for v in P.d]) for P in probs]).contiguous()
    a, b = _batch(probs), _batch(probs)
    for h in (a, b):
        h.set_variant(3, 4, 2)
    sa, sb = a.zero_batch_state(), b.zero_batch_state()
    n = probs[0].n
    c = (n - 1) / 2.0
    u = np.zeros((2, n, n), np.float32)
    u[1] = (-0.55 * (np.arange(n) - c))[:, None]   # pull-back compresses rows: q within ~2.2 px map near p
    gate = a.offsets[1] + 1                        # a gate of the field slice
    for e in range(3):
        if e == 1:
            for h in (a, b):
                h.set_motion(gate, ("field", torch.from_numpy(u).cuda()))
            assert a.info()["window_radius"] >= 2
        if e == 2:
            for h in (a, b):
                h.set_variant(0, 2, 1)
        seq = [g for sq in _seqs(probs, e) for g in sq]
        a.batch_spdhg_epoch(sa, d, alpha, sig, tau, th, p, seq, use_graph=True)
        b.batch_spdhg_epoch(sb, d, alpha, sig, tau, th, p, seq, use_graph=False)
        torch.cuda.synchronize()
        for k in ("x", "z", "zbar", "y"):
            assert torch.equal(sa[k], sb[k]), (e, k)
