"""Benchmark of the hot path: SPDHG epochs and A_i / A_i^* pairs on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

One step = one SPDHG epoch (N iterations of Algorithm 1: warp, projection
fused with the dual step, backprojection, transposed warp fused with the
z / z-bar / x updates) on synthetic data resident in device memory. Prints one
JSON line with the epoch rate, the A_i + A_i^* pair rate, the roofline of the
dominant kernel (per-launch durations from HIP events on the library's stream)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A_i+A_i^* pairs/sec and SPDHG epochs/sec at 512², N=16; HBM GB/s vs peak"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def joseph_nnz(n: int, na: int, nd: int) -> int:
    """Nonzero weights of the Joseph matrix (taps inside the image with a
    nonzero interpolation weight), counted angle by angle from the geometry."""
    half = (n - 1) / 2.0
    t = np.arange(nd) - (nd - 1) / 2.0
    pos = np.arange(n) - half
    total = 0
    for k in range(na):
        th = math.pi * k / na
        cs, sn = math.cos(th), math.sin(th)
        rows = 4 * k <= na or 4 * k >= 3 * na
        cf = ((t[None, :] - pos[:, None] * sn) / cs if rows else (t[None, :] - pos[:, None] * cs) / sn) + half
        c0 = np.floor(cf)
        f = cf - c0
        total += int(np.count_nonzero((c0 >= 0) & (c0 <= n - 1) & (f < 1.0)))
        total += int(np.count_nonzero((c0 + 1 >= 0) & (c0 + 1 <= n - 1) & (f > 0.0)))
    return total


def summary_fields(name: str, prefix: str, dominant: str, variant: dict):
    """The key=value fields of the line of a committed counter summary
    (profiles/<name>) that starts with `prefix` and names this kernel class
    and projector variant, or None when there is no such line or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    want = {"class": dominant, "fwd": str(variant.get("fwd")),
            "adj": f"{variant.get('adj_px')},{variant.get('adj_shares')}"}
    h = hashlib.sha256()
    for src in ("mcr_joseph_tiled.h", "mcr_kernels.h"):
        with open(os.path.join(ROOT, "paper_2410_10503_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    for line in open(path):
        if not line.startswith(prefix):
            continue
        fields = dict(tok.split("=", 1) for tok in line.split() if "=" in tok)
        if all(fields.get(k) == v for k, v in want.items()):
            if fields.get("sources_sha256_16") != h.hexdigest()[:16]:
                return None
            return fields
    return None


def measured_traffic(dominant: str, variant: dict):
    """HBM bytes per launch of the dominant kernel class from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE), or None (see summary_fields)."""
    f = summary_fields("traffic_joseph_pair_chest512_field16.md", "traffic: ", dominant, variant)
    return None if f is None else float(f["fetch_bytes"]) + float(f["write_bytes"])


def measured_valu_issue(dominant: str, variant: dict):
    """(fraction of the SIMD cycles on which the class's main kernel issued a
    VALU instruction, its wave-level VALU instructions per launch) from the
    committed SQ counter summary, or None (see summary_fields)."""
    f = summary_fields("sq_joseph_pair_chest512_field16.md", "sq: ", dominant, variant)
    return None if f is None else (float(f["valu_issue"]), float(f["valu_insts"]), f["kernel"])


ROOFS_SUMMARY = os.path.join(ROOT, "profiles", "roofs_mi355x.md")


def roofs_measurement():
    """On-chip and streaming roofs of the GPU from the probes of
    libmcr_probes.so (include/mcr_probes.h): LDS reads of 16-byte entries at
    conflict-free addresses (the projector pair's access), L2-resident
    16-byte global reads (2 MiB and 16 MiB buffers), and a 1 GiB device copy
    (read + write bytes). Each is the best of three runs."""
    import ctypes
    path = os.path.join(ROOT, "paper_2410_10503_amd", "libmcr_probes.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2410_10503_amd.build`")
    lib = ctypes.CDLL(path)
    lib.mcr_probe_lds_read.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.mcr_probe_l2_read.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.mcr_probe_copy.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]

    def best(fn, *args):
        vals = []
        for _ in range(3):
            v = ctypes.c_double()
            rc = fn(*args, ctypes.byref(v))
            if rc != 0:
                raise RuntimeError(f"{fn.__name__} failed with status {rc}")
            vals.append(v.value)
        return max(vals)

    out = {
        "lds_read_tbs": best(lib.mcr_probe_lds_read, 2048, 20000) / 1e12,
        "l2_read_tbs_2mib": best(lib.mcr_probe_l2_read, 2 << 20, 4096, 16) / 1e12,
        "l2_read_tbs_16mib": best(lib.mcr_probe_l2_read, 16 << 20, 4096, 4) / 1e12,
        "copy_gbs": best(lib.mcr_probe_copy, 1 << 30, 5) / 1e9,
        "probe": "lds: 2048 blocks x 256 threads x 80000 reads of 16 B; l2: 4096 blocks walking the buffer; "
                 "copy: 1 GiB, 5 repetitions",
    }
    return out


def lds_lanes_measurement():
    """Which lanes of a wave the LDS serves in one cycle for 16-byte reads,
    from the lane-pattern probe of libmcr_probes.so: octet i of the wave reads
    entries 0-7, octet j entries 16-23 (the same banks, other entries), every
    other octet entries 8-15. The read rate drops against the identity
    pattern (lane t reads entry t) exactly when octets i and j share a cycle.
    Then the quarter-turn projection's possible wave layouts, with the
    entries of lane (bin b, angle slot s) at floor(1.2 b + 0.5 s) (bins about
    1.2 entries apart, neighbouring angles half an entry)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2410_10503_amd", "libmcr_probes.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2410_10503_amd.build`")
    lib = ctypes.CDLL(path)
    lib.mcr_probe_lds_pattern.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]

    def rate(pattern):
        arr = (ctypes.c_int * 64)(*pattern)
        vals = []
        for _ in range(3):
            v = ctypes.c_double()
            rc = lib.mcr_probe_lds_pattern(arr, 2048, 5000, ctypes.byref(v))
            if rc != 0:
                raise RuntimeError(f"mcr_probe_lds_pattern failed with status {rc}")
            vals.append(v.value)
        return max(vals)

    base = rate(list(range(64)))
    pairs = {}
    for i in range(8):
        for j in range(i + 1, 8):
            pat = [(t & 7) + (0 if t >> 3 == i else 16 if t >> 3 == j else 8) for t in range(64)]
            pairs[f"{i},{j}"] = rate(pat) / base
    layouts = {
        "32 bins x 2 slots (bins 8k..8k+7 of slot 0, then of slot 1)":
            [((t & 7) | (((t >> 4) & 3) << 3), (t >> 3) & 1) for t in range(64)],
        "16 bins x 4 slots": [(t & 15, t >> 4) for t in range(64)],
        "8 bins x 8 slots (one slot per octet)": [(t & 7, t >> 3) for t in range(64)],
    }
    lay = {name: rate([int(1.2 * b + 0.5 * sl) for b, sl in lanes]) / base for name, lanes in layouts.items()}
    return {
        "identity_lds_read_tbs": base / 1e12,
        "octet_pairs_rate_vs_identity": pairs,
        "octet_pairs_served_together": sorted(k for k, v in pairs.items() if v < 0.85),
        "projection_wave_layouts_rate_vs_identity": lay,
        "probe": "2048 blocks x 256 threads x 4 x 5000 reads of 16 B per pattern, best of three",
    }


def measured_roofs():
    """The roofs line of the committed probe summary (profiles/), or None."""
    if not os.path.exists(ROOFS_SUMMARY):
        return None
    for line in open(ROOFS_SUMMARY):
        if line.startswith("roofs: "):
            return {k: float(v) for k, v in (tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)}
    return None


def _oracle_problem(name):
    """The oracle's gate operators and image of a workload (FP64)."""
    import synth
    from oracle.operators import GatedOperators
    wl = synth.WORKLOADS[name]
    params = wl.fields().astype(np.float64) if wl.motion == "field" else (
        wl.rigid() if wl.motion == "rigid" else None)
    ops = GatedOperators(wl.n, wl.n_angles, wl.n_det, wl.motion, params, n_gates=wl.n_gates)
    return wl, ops, np.asarray(wl.image(), dtype=np.float64)


def _oracle_iteration(args):
    """One SPDHG iteration of the oracle on gate g (a worker of the all-cores
    leg); returns its duration in seconds."""
    from oracle import spdhg
    name, g = args
    wl, ops, x = _oracle_problem(name)
    N = wl.n_gates
    st = spdhg.State.zeros(wl.n, N, wl.n_angles, wl.n_det)
    st.x = x
    d = [np.zeros((wl.n_angles, wl.n_det))] * N
    t0 = time.perf_counter()
    spdhg.iterate(ops, st, d, wl.alpha, [1e-3] * N, 1.0, 0.9, [1.0 / N] * N, [g])
    return time.perf_counter() - t0


def cpu_baseline(name: str):
    """The FP64 oracle (untuned, NumPy) on the workload, timed on the host's
    cores, before the GPU is touched: A_i x and A_i^* y on one core, one SPDHG
    iteration on one core, and one iteration per worker in as many worker
    processes as cores (up to 16, one gate each, all at once). Epochs/s are
    iterations/s over N (an epoch is N iterations)."""
    import multiprocessing as mp
    wl, ops, x = _oracle_problem(name)
    N = wl.n_gates
    g = N - 1
    t0 = time.perf_counter()
    s = ops.A(g, x)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    ops.At(g, s)
    t_adj = time.perf_counter() - t0
    t_it = _oracle_iteration((name, g))
    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")  # no GPU state exists yet in this process
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_iteration, [(name, (N - 1 - r) % N) for r in range(workers)], chunksize=1)
        t_all = time.perf_counter() - t0
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    all_eps = workers / t_all / N
    return {"value": all_eps, "unit": "SPDHG epochs/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} SPDHG iterations of the FP64 NumPy oracle at {wl.n}^2, {wl.n_angles}x{wl.n_det} "
                      f"(warp, projection, dual step, backprojection, transposed warp, updates), one per worker "
                      f"process on {workers} cores at once, {t_all:.1f} s wall; epochs/s = iterations/s / N",
            "one_core": {"epochs_per_s": 1.0 / (N * t_it), "s_per_iteration": t_it,
                         "s_apply_Ai": t_fwd, "s_apply_Ai_adjoint": t_adj,
                         "pairs_per_s": 1.0 / (t_fwd + t_adj)},
            "all_cores": {"workers": workers, "wall_s": t_all, "iterations_per_s": workers / t_all,
                          "epochs_per_s": all_eps},
            "host_cpus": os.cpu_count(), "cpu_model": cpu}


def copy_gbs(nbytes: int = 1 << 30, reps: int = 5):
    """Device-to-device copy rate (bytes read + written per second) of a
    buffer far larger than the on-chip caches: the achievable streaming rate
    the streaming kernels are compared with."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    rate = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3)
    del a, b
    return rate / 1e9


def batched_measurement(steps: int, seed: int = 4, variant=None, per_slice: bool = True):
    """64 independent 256^2 slices (360 x 366), gate counts uniform in {4..32},
    rigid and non-rigid motion alternating: epochs/s of the batched, graph-
    replayed epoch, of the same without the graph, and of the per-slice form
    (one handle per slice, epochs one after the other). Also the streaming
    rate of the step (i) and transposed-warp + update launches of one plain
    epoch (HIP events per launch) against the device copy rate."""
    import torch
    import synth
    from paper_2410_10503_amd import BatchHandle, Handle, step_sizes
    rng = np.random.default_rng(seed)
    S, n, na, nd = 64, 256, 360, 366
    ngs = [int(v) for v in rng.integers(4, 33, size=S)]
    motion, images = [], []
    for s_ in range(S):
        ng = ngs[s_]
        if s_ % 2:
            f = synth.dilatation_fields(n, ng, 100 + s_)
            motion += [("field", torch.from_numpy(f[i]).cuda()) for i in range(ng)]
        else:
            r = synth.rigid_params(ng, 100 + s_, 8.0, 10.0)
            motion += [("rigid", tuple(r[i])) for i in range(ng)]
        images.append(synth.ellipse_phantom(n, 200 + s_))
    bh = BatchHandle(n, na, nd, ngs, motion, dtype=torch.float32)
    G = sum(ngs)
    d = torch.empty((G, na, nd), dtype=torch.float32, device="cuda")
    for s_ in range(S):
        xg = torch.from_numpy(images[s_]).cuda()
        scale = 0.01 * float(bh.project(xg).abs().max()) / math.sqrt(ngs[s_])
        for k in range(ngs[s_]):
            gid = bh.offsets[s_] + k
            bh.apply_Ai(gid, xg, d[gid])
        noise = torch.from_numpy(synth.unit_noise((ngs[s_], na, nd), 300 + s_).astype(np.float32)).cuda()
        d[bh.offsets[s_]:bh.offsets[s_] + ngs[s_]] += scale * noise
    alpha = [1e-3] * S
    sig, tau, th, p = [], [], [], []
    for s_ in range(S):
        a, b, c, _ = step_sizes("spdhg", [2.0 * na * n] * ngs[s_], alpha[s_], ngs[s_])
        sig += a
        tau.append(b)
        th.append(c)
        p += [1.0 / ngs[s_]] * ngs[s_]
    # the batched launches cover the slices still iterating (S at the first
    # step, fewer later): tune for the mean number of slices per launch
    if variant is None:
        variant = bh.autotune(max(1, round(G / max(ngs))))
    else:
        bh.set_variant(variant["fwd"], variant["adj_px"], variant["adj_shares"])

    def seqs(e):
        return [int(g) for s_ in range(S) for g in synth.gate_sequence(ngs[s_], 500 + s_, e)]

    out = {"workload": f"{S} slices of {n}^2, {na}x{nd}, gates U{{4..32}} (sum {G}), rigid/field alternating",
           "gate_iterations_per_epoch": G, "projector_variant": variant}
    for use_graph in (True, False):
        st = bh.zero_batch_state()
        bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, seqs(0), use_graph=use_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(steps):
            bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, seqs(1 + e), use_graph=use_graph)
        torch.cuda.synchronize()
        out["epochs_per_s_graph" if use_graph else "epochs_per_s_plain"] = steps / (time.perf_counter() - t0)
    # streaming launches of one plain epoch: step (i) of all slices reads x
    # and z-bar and writes x (3 images per slice); the transposed warp +
    # update of a gate iteration reads b and z and writes z and z-bar (4
    # images), plus x read and written except at a slice's last iteration,
    # plus the two field planes of a field gate. The images of the 64 slices
    # (17 MB per array) may be served from the 256 MB last-level cache.
    bh.profile(True)
    bh.profile_read()
    bh.batch_spdhg_epoch(st, d, alpha, sig, tau, th, p, seqs(1 + steps), use_graph=False)
    ks = bh.profile_read()
    bh.profile(False)
    img_b = 4.0 * n * n
    g_field = sum(ngs[s_] for s_ in range(S) if s_ % 2)
    copy_rate = copy_gbs()
    stream = {"copy_gbs": copy_rate}
    for name, nbytes in (("xstep", 3 * S * img_b), ("twarp", img_b * (4 * G + 2 * (G - S) + 2 * g_field))):
        ms, cnt = ks[name]
        if cnt:
            gbs = nbytes / (ms / 1e3) / 1e9
            stream[name] = {"launches": cnt, "us_per_launch": 1e3 * ms / cnt, "bytes_per_epoch": nbytes,
                            "gbs": gbs, "frac_of_copy": gbs / copy_rate, "frac_of_peak": gbs / PEAK_HBM_GBS}
    out["streaming"] = stream
    if not per_slice:
        bh.close()
        return out
    # per-slice form: one handle per slice, same kernels and variant
    handles = []
    for s_ in range(S):
        h = Handle(n, na, nd, motion[bh.offsets[s_]:bh.offsets[s_] + ngs[s_]], dtype=torch.float32)
        h.set_variant(variant["fwd"], variant["adj_px"], variant["adj_shares"])
        dd = [d[bh.offsets[s_] + k] for k in range(ngs[s_])]
        handles.append((h, h.zero_state(), dd))

    def per_slice_epoch(e):
        sq = seqs(e)
        for s_, (h, st_, dd) in enumerate(handles):
            o = bh.offsets[s_]
            h.spdhg_epoch(st_, dd, alpha[s_], sig[o:o + ngs[s_]], tau[s_], th[s_], p[o:o + ngs[s_]],
                          sq[o:o + ngs[s_]])

    per_slice_epoch(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(steps):
        per_slice_epoch(1 + e)
    torch.cuda.synchronize()
    out["epochs_per_s_per_slice"] = steps / (time.perf_counter() - t0)
    for h, _, _ in handles:
        h.close()
    bh.close()
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden")


def hip_data(n, na, nd, kind, params, x_true, noise, hashes=None):
    """Gated data d_i = A_i x_true + (s / sqrt(N)) noise_i in float32, with
    s = 0.01 max|A x_true| (Section II-A), the ray sums taken from the
    library's FP64 path. With `hashes` (the SHA-256 of the FP64 oracle's
    float32 data, stored beside its results) each gate is checked against
    them: returns (d, gates whose bytes differ). The two FP64 ray sums differ
    by ~1e-16 relative, so a gate differs only where a value sits next to a
    float32 rounding tie, by one unit in the last place."""
    import hashlib
    import torch
    from paper_2410_10503_amd import Handle
    N = noise.shape[0]
    if kind == "rigid":
        motion = [("rigid", tuple(float(v) for v in params[i])) for i in range(N)]
    else:
        ft = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
        motion = [("field", ft[i].contiguous()) for i in range(N)]
    h = Handle(n, na, nd, motion, dtype=torch.float64)
    xd = torch.from_numpy(np.asarray(x_true, dtype=np.float64)).cuda()
    scale = 0.01 * float(np.max(np.abs(h.project(xd).cpu().numpy())))
    d, differ = [], []
    for i in range(N):
        v32 = (h.apply_Ai(i, xd).cpu().numpy() + (scale / math.sqrt(N)) * noise[i]).astype(np.float32)
        if hashes is not None and hashlib.sha256(v32.tobytes()).hexdigest() != str(hashes[i]):
            differ.append(i)
        d.append(v32)
    h.close()
    return d, differ


def pdhg_spdhg_measurement(epochs: int = 10):
    """PDHG against SPDHG on the 512^2 rigid workload (8 gates, 720 x 730,
    FP32): epochs/s of each (a PDHG epoch is one iteration over all gates,
    launched 8 gates wide; an SPDHG epoch 8 one-gate iterations), and, where
    the FP64 oracle's stored 50-epoch iterates are present
    (tests/golden/fullsize_c2_*.npz), the float32 iterates after 50 epochs
    from zero against them, on the same data (hash-checked), step sizes and
    gate draws: relative L2 and largest entry error over the largest entry."""
    import torch
    import synth
    from paper_2410_10503_amd import Handle, step_sizes
    wl = synth.WORKLOADS["ellipses512_rigid8"]
    N = wl.n_gates
    params = wl.rigid()
    motion = [("rigid", tuple(params[i])) for i in range(N)]
    h = Handle(wl.n, wl.n_angles, wl.n_det, motion, dtype=torch.float32)
    noise = synth.unit_noise((N, wl.n_angles, wl.n_det), wl.noise_seed)
    gold = {}
    for algo in ("spdhg", "pdhg"):
        path = os.path.join(GOLDEN, f"fullsize_c2_{algo}.npz")
        if os.path.exists(path):
            z = np.load(path)
            gold[algo] = (z, json.loads(str(z["meta"])))
    hashes = gold["spdhg"][0]["d_sha256"] if "spdhg" in gold else None
    d32, differ = hip_data(wl.n, wl.n_angles, wl.n_det, "rigid", params, wl.image(), noise, hashes)
    data = [torch.from_numpy(v).cuda() for v in d32]
    v0 = torch.from_numpy(synth.random_image(wl.n, 17).astype(np.float64)).cuda()
    norms = [h.power_norm_sq(i, v0, max_iter=25, rtol=1e-6)[0] for i in range(N)]
    stacked = h.power_norm_sq(-1, v0, max_iter=25, rtol=1e-6)[0]
    steps = {"spdhg": step_sizes("spdhg", norms, wl.alpha, N), "pdhg": step_sizes("pdhg", [stacked], wl.alpha, N)}
    out = {"workload": f"{wl.name}: {wl.n}^2, {wl.n_angles}x{wl.n_det}, {N} rigid gates, float32"}

    def epoch(st, algo, e, sig, tau, th):
        if algo == "pdhg":
            h.pdhg_epoch(st, data, wl.alpha, sig, tau, th)
        else:
            h.spdhg_epoch(st, data, wl.alpha, sig, tau, th, [1.0 / N] * N, synth.gate_sequence(N, wl.gate_seed, e))

    for algo in ("pdhg", "spdhg"):
        variant = h.autotune(N if algo == "pdhg" else 1)  # launches 8 gates or one gate wide
        sig, tau, th, rate = steps[algo]
        st = h.zero_state()
        for e in range(5):
            epoch(st, algo, e, sig, tau, th)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(epochs):
            epoch(st, algo, 5 + e, sig, tau, th)
        torch.cuda.synchronize()
        res = {"epochs_per_s": epochs / (time.perf_counter() - t0), "projector_variant": variant,
               "per_epoch_rate": rate}
        if algo in gold:
            z, meta = gold[algo]
            st = h.zero_state()
            for e in range(50):
                epoch(st, algo, e, meta["sigma"], meta["tau"], meta["theta"])
            errs = {}
            for name, t in (("x", st.x), ("zbar", st.zbar)):
                a, b = t.double().cpu().numpy(), z[f"e50_{name}"]
                errs[name] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                              "rel_max": float(np.abs(a - b).max() / np.abs(b).max())}
            res["vs_fp64_oracle_after_50_epochs"] = errs
            res["data_gates_differing_from_the_oracle_in_the_last_bit"] = differ
        out[algo] = res
    h.close()
    return out


def autograd_measurement(reps: int = 3):
    """Differentiation through 10 unrolled SPDHG iterations at 512^2, 720 x 730,
    16 rigid gates: the plain 10 iterations against the checkpointed forward
    plus the reverse pass (image and 48 motion gradients)."""
    import torch
    import synth
    from paper_2410_10503_amd import Handle, step_sizes
    from paper_2410_10503_amd.autograd import unrolled_spdhg
    wl = synth.WORKLOADS["ellipses512_rigid16"]
    N = wl.n_gates
    params = wl.rigid()
    h = Handle(wl.n, wl.n_angles, wl.n_det, [("rigid", tuple(params[i])) for i in range(N)], dtype=torch.float32)
    h.autotune(1)
    xg = torch.from_numpy(wl.image()).cuda()
    d = [h.apply_Ai(i, xg) for i in range(N)]
    sigma, tau, theta, _ = step_sizes("spdhg", [3.7e5] * N, wl.alpha, N)
    p = [1.0 / N] * N
    seq = [int(g) for g in synth.gate_sequence(N, wl.gate_seed, 0, length=10)]
    x0 = (0.8 * xg).contiguous()
    mot = torch.tensor(params, dtype=torch.float64, device="cuda")

    def plain():
        st = h.zero_state()
        st.x.copy_(x0)
        h.spdhg_iterate(st, d, wl.alpha, sigma, tau, theta, p, seq)
        return st.x

    def with_grad():
        xr = x0.clone().requires_grad_(True)
        mr = mot.clone().requires_grad_(True)
        xk = unrolled_spdhg(h, xr, mr, d, wl.alpha, sigma, tau, theta, p, seq)
        torch.sum((xk - xg) ** 2).backward()
        return xr.grad

    out = {"workload": "10 unrolled SPDHG iterations, 512^2, 720x730, 16 rigid gates, gradients w.r.t. "
                       "the start image and 48 rigid parameters"}
    for name, fn in (("plain_forward_ms", plain), ("forward_and_backward_ms", with_grad)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name] = 1e3 * (time.perf_counter() - t0) / reps
    out["ratio"] = out["forward_and_backward_ms"] / out["plain_forward_ms"]
    # the library's launches alone (HIP events around each), against the wall
    # time above (which also holds the host work of the autograd function)
    for name, fn in (("plain_forward_kernel_ms", plain), ("forward_and_backward_kernel_ms", with_grad)):
        h.profile(True)
        h.profile_read()
        fn()
        torch.cuda.synchronize()
        out[name] = sum(v[0] for v in h.profile_read().values())
        h.profile(False)
    h.close()
    return out


def registration_measurement():
    """Rigid registration (the preliminary step of Section I) of the 16 gate
    images of the 512^2 rigid workload to the reference image, each from zero:
    the gate images are the reference warped by the workload's motion."""
    import torch
    import synth
    from paper_2410_10503_amd import Handle
    wl = synth.WORKLOADS["ellipses512_rigid16"]
    N = wl.n_gates
    params = wl.rigid()
    h = Handle(wl.n, wl.n_angles, wl.n_det, [("rigid", tuple(params[i])) for i in range(N)], dtype=torch.float32)
    ref = torch.from_numpy(wl.image()).cuda()
    targets = [h.warp(i, ref).clone() for i in range(N)]
    torch.cuda.synchronize()
    scale = np.array([(wl.n - 1) / 2.0, 1.0, 1.0])
    t0 = time.perf_counter()
    res = [h.register_rigid(i, ref, targets[i], max_iter=300, tol=1e-5) for i in range(N)]
    dt = time.perf_counter() - t0
    err = max(float(np.abs((np.array(th) - params[i]) * scale).max()) for i, (th, _, _) in enumerate(res))
    h.close()
    out = {"workload": "16 rigid gates at 512^2 (rotations up to 8 deg, shifts up to 10 px), each gate image "
                       "registered to the reference from zero, float32",
           "ms_per_gate": 1e3 * dt / N, "steps_mean": float(np.mean([k for _, _, k in res])),
           "max_error_px": err}
    # the chest experiment's motion kind: 10 gates of vertical linear
    # dilatation (up to 8 px at the edge) plus small shifts, as affine fields
    # (the gate images: the reference warped by the library with each field)
    Nf = 10
    n = wl.n
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64) - c
    thetas = [(0.0, 0.0, 0.0, 8.0 * (i / 9.0) / c, 0.5 * i / 9.0, -0.7 * i / 9.0) for i in range(Nf)]
    fields = [torch.from_numpy(np.stack([(t[0] * xx + t[1] * yy) + t[4], (t[2] * xx + t[3] * yy) + t[5]])
                               .astype(np.float32)).cuda() for t in thetas]
    hf = Handle(n, wl.n_angles, wl.n_det, [("field", f) for f in fields], dtype=torch.float32)
    targets = [hf.warp(i, ref).clone() for i in range(Nf)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [hf.register_affine(i, ref, targets[i], max_iter=500, tol=1e-5) for i in range(Nf)]
    dt = time.perf_counter() - t0
    sa = np.array([c] * 4 + [1.0, 1.0])
    err = max(float(np.abs((np.array(th) - np.array(thetas[i])) * sa).max()) for i, (th, _, _) in enumerate(res))
    hf.close()
    out["affine"] = {"workload": "10 field gates at 512^2, vertical linear dilatations up to 8 px plus shifts, "
                                 "affine registration from zero, float32",
                     "ms_per_gate": 1e3 * dt / Nf, "steps_mean": float(np.mean([k for _, _, k in res])),
                     "max_error_px": err}
    # dense fields: the headline workload's own displacement fields (vertical
    # dilatation plus Gaussian bumps), gates 4, 8, 12, 15, each registered from
    # zero, one level of 300 steps and a coarse-to-fine schedule (widths 8, 4,
    # 2, 1, 0 px, 150 steps each), lambda = 0.1; error over the pixels where
    # the chest phantom has an edge
    try:
        out["dense"] = dense_registration_measurement(n)
    except RuntimeError as e:  # a result the transposed warp's window rejects
        out["dense"] = {"error": str(e)}
    return out


def dense_registration_measurement(n: int):
    import torch
    import synth
    from paper_2410_10503_amd import Handle
    wc = synth.WORKLOADS["chest512_field16"]
    true_f = wc.fields()
    gates = [4, 8, 12, 15]
    hd = Handle(n, wc.n_angles, wc.n_det, [("field", torch.from_numpy(true_f[i]).cuda()) for i in gates],
                dtype=torch.float32)
    xc = torch.from_numpy(wc.image()).cuda()
    targets = [hd.warp(j, xc).clone() for j in range(len(gates))]
    torch.cuda.synchronize()
    E0 = [hd.register_field(j, xc, targets[j], lam=0.1, max_iter=0)[1] for j in range(len(gates))]
    img = wc.image()
    edge = np.hypot(*np.gradient(img)) > 0
    errs0 = [float(np.sqrt(np.mean(np.sum(true_f[g].astype(np.float64) ** 2, axis=0)[edge]))) for g in gates]
    out = {"workload": "gates 4, 8, 12, 15 of chest512_field16 (dilatation + Gaussian bumps), dense field "
                       "registration from zero, lambda 0.1, float32", "rms_true_field_px_at_edges": errs0}
    for name, sig, steps in (("one_level", (), 300), ("coarse_to_fine", (8.0, 4.0, 2.0, 1.0, 0.0), 150)):
        t0 = time.perf_counter()
        res = [hd.register_field(j, xc, targets[j], field=torch.zeros(2, n, n, device="cuda"), lam=0.1,
                                 max_iter=steps, tol=1e-3, sigmas=sig) for j in range(len(gates))]
        dt = time.perf_counter() - t0
        errs = [float(np.sqrt(np.mean(np.sum((u.cpu().numpy() - true_f[g]) ** 2, axis=0)[edge])))
                for (u, _, _), g in zip(res, gates)]
        # the coarse-to-fine energy is that of the last (unsmoothed) level
        out[name] = {"sigmas": list(sig), "max_steps_per_level": steps, "ms_per_gate": 1e3 * dt / len(gates),
                     "steps_mean": float(np.mean([k for _, _, k in res])),
                     "energy_ratio_mean": float(np.mean([r[1] / e0 for r, e0 in zip(res, E0)])),
                     "rms_error_px_at_edges": errs}
    hd.close()
    return out


def subsets_measurement(h, d, wl, gate_norms, v0, gate_eps: float, variant: dict, M: int = 4, epochs: int = 10):
    """Sampling over gates x angle subsets (the next step named in the
    Conclusions) on the same handle and data, for M contiguous angle subsets
    and for M paired ones (a range of the first half of the angles with its
    partners a quarter turn away, which the quarter-turn projector pair
    serves): N M blocks, an epoch of N M block iterations (the operator work
    of one PDHG iteration). Reports epochs/s, the theoretical per-epoch rates
    l(kappa, N M) against the gate-only l(kappa, N) at the workload's alpha
    and in the paper's regime (kappa = |A|^2 / alpha = 70), and the
    contraction per second, epochs/s x ln(rate), against the gate epochs'
    (gate_eps: the gate-only epochs/s of the same handle, with the projector
    variants `variant`)."""
    import torch
    import synth
    from paper_2410_10503_amd import step_sizes_blocks
    N = h.n_gates
    nb = N * M

    def l(kappa, n):
        return (1.0 - 2.0 / (n * (1.0 + math.sqrt(1.0 + kappa)))) ** n

    a70 = max(gate_norms) / 70.0
    r_g = l(max(gate_norms) / (wl.alpha * N), N)
    r_g70 = l(max(gate_norms) / (a70 * N), N)
    out = {"workload": f"{wl.name} with {M} angle subsets ({nb} blocks), epoch = {nb} block iterations",
           "gates": {"epochs_per_s": gate_eps, "rate_per_epoch": r_g, "rate_per_epoch_kappa70": r_g70,
                     "contraction_per_s": gate_eps * math.log(r_g),
                     "contraction_per_s_kappa70": gate_eps * math.log(r_g70)}}
    base = (variant["fwd"], variant["adj_px"], variant["adj_shares"])
    for partition in ("contiguous", "paired"):
        h.set_subsets(M, paired=partition == "paired")
        bnorms = [h.block_norm_sq(b // M, b % M, v0, max_iter=15, rtol=1e-5)[0] for b in range(nb)]
        sig, tau, th, rate_b = step_sizes_blocks(bnorms, wl.alpha, N, M)
        p = [1.0 / nb] * nb
        st = h.zero_state()

        def epoch(e):
            h.spdhg_blocks_iterate(st, d, wl.alpha, sig, tau, th, p, synth.gate_sequence(nb, wl.gate_seed, e))

        # a block launch holds 1/M of the angles: the adjoint's angle shares
        # are chosen among a few counts for it (the gate launches keep theirs)
        times = {}
        for shares in sorted({base[2], max(1, base[2] // M), max(1, base[2] // 2), 2 * base[2] // M,
                              max(1, 3 * base[2] // 4)}):
            h.set_variant(base[0], base[1], min(16, shares))
            epoch(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for e in range(epochs):
                epoch(1 + e)
            torch.cuda.synchronize()
            times[min(16, shares)] = time.perf_counter() - t0
        best = min(times, key=times.get)
        el = times[best]
        eps = epochs / el
        r70 = l(max(bnorms) / (a70 * N), nb)
        out[partition] = {
            "epochs_per_s": eps, "us_per_block_iteration": 1e6 * el / (epochs * nb), "adjoint_shares": best,
            "us_per_block_iteration_by_shares": {str(k): 1e6 * v / (epochs * nb) for k, v in sorted(times.items())},
            "block_norm_sq_range": [min(bnorms), max(bnorms)],
            "rate_per_epoch": rate_b, "rate_per_epoch_kappa70": r70,
            "contraction_per_s": eps * math.log(rate_b), "contraction_per_s_kappa70": eps * math.log(r70)}
    h.set_variant(*base)
    h.set_subsets(1)
    return out


def subsets_block_measurement(M: int, epochs: int, variant=None):
    """The block iterations of M paired angle subsets alone, on the headline
    workload (for kernel traces of the subset launches, which the bench's
    subsets measurement mixes with the gate epochs): block norms by power
    iteration, step sizes, one untimed epoch of N M block iterations, then
    `epochs` timed ones, with the projector variants given (else autotuned
    for one gate per launch)."""
    import torch
    import synth
    from paper_2410_10503_amd import Handle, step_sizes_blocks
    wl = synth.WORKLOADS["chest512_field16"]
    dev = torch.device("cuda:0")
    n, na, nd, N = wl.n, wl.n_angles, wl.n_det, wl.n_gates
    fields = wl.fields()
    h = Handle(n, na, nd, [("field", torch.from_numpy(fields[i]).to(dev)) for i in range(N)],
               dtype=torch.float32, device=dev)
    xg = torch.from_numpy(wl.image()).to(dev)
    d = [h.apply_Ai(i, xg) for i in range(N)]
    if variant:
        h.set_variant(variant["fwd"], variant["adj_px"], variant["adj_shares"])
    else:
        variant = h.autotune(1)
    h.set_subsets(M, paired=True)
    nb = N * M
    v0 = torch.from_numpy(synth.random_image(n, 17).astype(np.float64)).to(dev)
    bnorms = [h.block_norm_sq(b // M, b % M, v0, max_iter=15, rtol=1e-5)[0] for b in range(nb)]
    sig, tau, th, rate = step_sizes_blocks(bnorms, wl.alpha, N, M)
    p = [1.0 / nb] * nb
    st = h.zero_state()

    def epoch(e):
        h.spdhg_blocks_iterate(st, d, wl.alpha, sig, tau, th, p, synth.gate_sequence(nb, wl.gate_seed, e))

    epoch(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(epochs):
        epoch(1 + e)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.close()
    return {"workload": f"{wl.name}, {M} paired angle subsets ({nb} blocks), epoch = {nb} block iterations",
            "projector_variant": variant, "epochs": epochs, "epochs_per_s": epochs / el,
            "us_per_block_iteration": 1e6 * el / (epochs * nb), "rate_per_epoch": rate}


def paper_experiment(epochs: int = 30, seeds: int = 8, reference=None):
    """Section III on the GPU in FP64: l2^2-distance to the saddle point per
    epoch for PDHG and SPDHG (mean over seeds) against Theorem 1's rates, in
    the paper's regime kappa = |A|^2 / alpha = 70, with 20 rigid gates and 10
    dilatation gates (synthetic stand-ins for the walnut and chest data); and
    the motion-compensated minimiser against the one without motion
    compensation (D_i = I, same data). The saddle point is the linear solve
    (alpha I + N^-1 sum A_i^* A_i) x = N^-1 sum A_i^* d_i by conjugate
    gradients on the library's FP64 operators.

    reference (optional, per problem name): {"alpha", "d", "xs", "ys",
    "xs_nomc"}, the FP64 oracle's step parameter, data and minimisers (the
    tests build it from the stored oracle results); given, the runs use its
    alpha and data and measure distances to its (x*, y*), and the
    conjugate-gradient minimisers are compared with its own. Without it the
    stored oracle minimisers (tests/golden/fullsize_k70.npz), when present,
    are only compared with the conjugate-gradient ones."""
    import torch
    import synth
    from paper_2410_10503_amd import Handle, step_sizes
    dt = torch.float64
    out = {}
    for name in ("ellipses128_rigid20_k70", "chest128_field10_k70"):
        wl = synth.WORKLOADS[name]
        n, na, nd, N = wl.n, wl.n_angles, wl.n_det, wl.n_gates
        if wl.motion == "rigid":
            motion = [("rigid", tuple(r)) for r in wl.rigid()]
        else:
            f = torch.from_numpy(wl.fields()).cuda()
            motion = [("field", f[i].contiguous()) for i in range(N)]
        h = Handle(n, na, nd, motion, dtype=dt)
        plain = Handle(n, na, nd, ["identity"] * N, dtype=dt)
        v0 = torch.from_numpy(synth.random_image(n, 17).astype(np.float64)).cuda()
        normA, _ = plain.power_norm_sq(0, v0, max_iter=500, rtol=1e-12)
        rf = reference.get(name) if reference else None
        alpha = rf["alpha"] if rf else normA / wl.kappa
        xt = torch.from_numpy(wl.image().astype(np.float64)).cuda()
        if rf:
            d = [torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda() for v in rf["d"]]
        else:
            ref = plain.project(xt)
            scale = 0.01 * float(ref.abs().max()) / math.sqrt(N)
            noise = torch.from_numpy(synth.unit_noise((N, na, nd), wl.noise_seed)).cuda()
            d = [h.apply_Ai(i, xt) + scale * noise[i] for i in range(N)]

        def solve(hh):
            def normal(v):
                acc = alpha * v
                for i in range(N):
                    acc = acc + hh.apply_Ai_adjoint(i, hh.apply_Ai(i, v)) / N
                return acc
            rhs = sum(hh.apply_Ai_adjoint(i, d[i]) for i in range(N)) / N
            x = torch.zeros_like(rhs)
            r = rhs.clone()
            pdir = r.clone()
            rr = float((r * r).sum())
            b2 = float((rhs * rhs).sum())
            it = 0
            for it in range(1, 2001):
                ap = normal(pdir)
                a = rr / float((pdir * ap).sum())
                x = x + a * pdir
                r = r - a * ap
                rr_new = float((r * r).sum())
                if rr_new <= 1e-26 * b2:
                    break
                pdir = r + (rr_new / rr) * pdir
                rr = rr_new
            return x, it

        xs_cg, cg_it = solve(h)
        if rf:
            xs = torch.from_numpy(np.asarray(rf["xs"], dtype=np.float64)).cuda()
            ys = [torch.from_numpy(np.asarray(v, dtype=np.float64)).cuda() for v in rf["ys"]]
        else:
            xs = xs_cg
            ys = [(2.0 / N) * (h.apply_Ai(i, xs) - d[i]) for i in range(N)]

        def dist2(st):
            return float(((st.x - xs) ** 2).sum()) + sum(float(((a - b) ** 2).sum()) for a, b in zip(st.y, ys))

        gn = [h.power_norm_sq(i, v0, max_iter=500, rtol=1e-12)[0] for i in range(N)]
        sn, _ = h.power_norm_sq(-1, v0, max_iter=500, rtol=1e-12)
        k_s, k_p = max(gn) / (alpha * N), sn / (alpha * N)

        def l(kappa, m):
            return (1.0 - 2.0 / (m * (1.0 + math.sqrt(1.0 + kappa)))) ** m

        sig, tau, th, rate_p = step_sizes("pdhg", [sn], alpha, N)
        st = h.zero_state()
        dp = []
        for e in range(epochs):
            h.pdhg_epoch(st, d, alpha, sig, tau, th)
            dp.append(dist2(st))
        sig, tau, th, rate_s = step_sizes("spdhg", gn, alpha, N)
        runs = []
        for seed in range(seeds):
            st = h.zero_state()
            cur = []
            for e in range(epochs):
                h.spdhg_epoch(st, d, alpha, sig, tau, th, [1.0 / N] * N, synth.gate_sequence(N, seed, e))
                cur.append(dist2(st))
            runs.append(cur)
        ds = np.mean(runs, axis=0)

        def fitted(series):
            e0 = 5
            return float(math.exp(np.polyfit(np.arange(e0, epochs), np.log(np.asarray(series)[e0:]), 1)[0]))

        xnm, _ = solve(plain)
        err = lambda a: float(torch.linalg.norm(a - xt) / torch.linalg.norm(xt))  # noqa: E731
        # the oracle's minimisers: the reference, else the stored results
        oracle = None
        if rf:
            oracle = {"alpha": rf["alpha"], "xs": rf["xs"], "xs_nomc": rf["xs_nomc"], "source": "reference"}
        else:
            path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "fullsize_k70.npz")
            if os.path.exists(path):
                z = np.load(path)
                key = name.split("_")[1]
                pm = json.loads(str(z["meta"]))["problems"][name]
                oracle = {"alpha": pm["alpha"], "xs": z[f"{key}_xs"], "xs_nomc": z[f"{key}_xs_nomc"],
                          "source": "tests/golden/fullsize_k70.npz"}
        vs_oracle = None
        if oracle is not None:
            rel_np = lambda a, b: float(np.linalg.norm(a.cpu().numpy() - b) / np.linalg.norm(b))  # noqa: E731
            xo = torch.from_numpy(np.asarray(oracle["xs"], dtype=np.float64)).cuda()
            xo_nm = torch.from_numpy(np.asarray(oracle["xs_nomc"], dtype=np.float64)).cuda()
            vs_oracle = {"source": oracle["source"], "alpha_rel": abs(alpha - oracle["alpha"]) / oracle["alpha"],
                         "xs_cg_rel": rel_np(xs_cg, oracle["xs"]), "xs_nomc_cg_rel": rel_np(xnm, oracle["xs_nomc"]),
                         "rel_error_vs_truth": {"motion_compensated": err(xo), "no_motion_compensation": err(xo_nm)}}
        out[name] = {
            "n": n, "n_angles": na, "n_det": nd, "gates": N, "motion": wl.motion, "alpha": alpha,
            "norm_A_sq": normA, "kappa_spdhg": k_s, "kappa_pdhg": k_p,
            "gate_norm_ratio_max": max(gn) / normA, "stacked_norm_ratio": sn / (N * normA),
            "cg_iterations": cg_it,
            "rate_per_epoch": {"pdhg_theory": l(k_p, 1), "pdhg_observed": fitted(dp),
                               "spdhg_theory": l(k_s, N), "spdhg_observed_mean": fitted(ds)},
            "dist_sq_pdhg": dp, "dist_sq_spdhg_mean": [float(v) for v in ds],
            "rel_error_vs_truth": {"motion_compensated": err(xs_cg), "no_motion_compensation": err(xnm)},
            "oracle_minimisers": vs_oracle,
        }
        log(f"{name}: {json.dumps({k: v for k, v in out[name].items() if not k.startswith('dist_sq')})}")
        h.close()
        plain.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 20 warm-up epochs (about 30 ms) bring the GPU to its sustained clocks
    # before the timed region: with 2, the first timed epochs run ~5% slower
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="chest512_field16")
    ap.add_argument("--pairs", type=int, default=160)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64 x 256^2 measurement")
    ap.add_argument("--no-autograd", action="store_true", help="skip the differentiation measurement")
    ap.add_argument("--no-subsets", action="store_true", help="skip the gates x angle-subsets measurement")
    ap.add_argument("--subsets-m", default="4",
                    help="comma-separated subset counts M of the subsets measurement (the first is reported "
                         "as 'subsets', the others as 'subsets_m<M>')")
    ap.add_argument("--no-registration", action="store_true", help="skip the rigid-registration measurement")
    ap.add_argument("--no-pdhg", action="store_true", help="skip the PDHG vs SPDHG measurement")
    ap.add_argument("--variant", default=None,
                    help="fwd,adj_px,adj_shares: use these projector variants instead of autotuning "
                         "(counter runs serialise dispatches, which would change the autotuner's choice)")
    ap.add_argument("--experiment",
                    choices=["paper", "batched", "subsets", "autograd", "registration", "pdhg", "roofs",
                             "lds-lanes"],
                    default=None,
                    help="paper: the Section III reproduction (rates vs Theorem 1, MC vs no-MC); batched: the "
                         "64-slice batched workload alone (--steps epochs, --variant applies), for counter "
                         "runs; subsets: the block iterations of the first --subsets-m paired subsets alone "
                         "(--steps epochs, --variant applies), for kernel traces; autograd, registration, pdhg: that measurement of the bench alone; roofs: the "
                         "LDS, L2 and copy probes; lds-lanes: the LDS lane-grouping probe; each instead of the "
                         "bench")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also copy 256 MiB once (reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "a design in the documentation, not a measured path.", file=sys.stderr)
        sys.exit(2)

    if args.experiment == "paper":
        print(json.dumps({"experiment": "section III reproduction", "results": paper_experiment()}), flush=True)
        return
    if args.experiment in ("autograd", "registration", "pdhg", "roofs", "lds-lanes"):
        fn = {"autograd": autograd_measurement, "registration": registration_measurement,
              "pdhg": pdhg_spdhg_measurement, "roofs": roofs_measurement,
              "lds-lanes": lds_lanes_measurement}[args.experiment]
        print(json.dumps({"experiment": args.experiment, "results": fn()}), flush=True)
        return
    if args.experiment == "subsets":
        v = None
        if args.variant:
            f, px, sh = (int(t) for t in args.variant.split(","))
            v = {"fwd": f, "adj_px": px, "adj_shares": sh}
        res = subsets_block_measurement(int(args.subsets_m.split(",")[0]), args.steps, variant=v)
        print(json.dumps({"experiment": "subsets", "results": res}), flush=True)
        return
    if args.experiment == "batched":
        v = None
        if args.variant:
            f, px, sh = (int(t) for t in args.variant.split(","))
            v = {"fwd": f, "adj_px": px, "adj_shares": sh}
        res = batched_measurement(args.steps, variant=v, per_slice=False)
        print(json.dumps({"experiment": "batched", "results": res}), flush=True)
        return

    # the CPU oracle first, on the host's cores, while no GPU state exists
    cpu_leg = None
    if not args.no_cpu:
        log("timing the FP64 CPU oracle (one core, then all cores) ...")
        cpu_leg = cpu_baseline(args.workload)
        log(f"cpu baseline: {cpu_leg}")

    import torch
    import synth
    from paper_2410_10503_amd import Handle, step_sizes

    wl = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, na, nd, N = wl.n, wl.n_angles, wl.n_det, wl.n_gates
    log(f"workload {wl.name}: {n}^2, {na}x{nd}, {N} {wl.motion} gates")

    x_true = wl.image()
    if wl.motion == "field":
        params = wl.fields()
        motion = [("field", torch.from_numpy(params[i]).to(dev)) for i in range(N)]
    elif wl.motion == "rigid":
        params = wl.rigid()
        motion = [("rigid", tuple(params[i])) for i in range(N)]
    else:
        params = None
        motion = ["identity"] * N
    h = Handle(n, na, nd, motion, dtype=torch.float32, device=dev)
    xg = torch.from_numpy(x_true).to(dev)

    # gated data d_i = A_i x + noise (Section II-A), generated on the device
    ref = h.project(xg)
    scale = 0.01 * float(ref.abs().max()) / math.sqrt(N)
    noise = torch.from_numpy(synth.unit_noise((N, na, nd), wl.noise_seed).astype(np.float32)).to(dev)
    d = [h.apply_Ai(i, xg) + scale * noise[i] for i in range(N)]
    del noise

    # step sizes from FP64 power-iteration norms (on the device)
    v0 = torch.from_numpy(synth.random_image(n, 17).astype(np.float64)).to(dev)
    norms = [h.power_norm_sq(i, v0, max_iter=25, rtol=1e-6)[0] for i in range(N)]
    sigma, tau, theta, rate = step_sizes("spdhg", norms, wl.alpha, N)
    p = [1.0 / N] * N
    log(f"|A_i|^2 in [{min(norms):.4g}, {max(norms):.4g}], per-epoch rate {rate:.6f}")

    if args.variant:
        f, px, sh = (int(v) for v in args.variant.split(","))
        h.set_variant(f, px, sh)
        variant = {"fwd": f, "adj_px": px, "adj_shares": sh}
        log(f"projector variants (fixed): {variant}")
    else:
        variant = h.autotune(1)
        log(f"autotuned projector variants: {variant}")
    st = h.zero_state()

    def epoch(e):
        h.spdhg_epoch(st, d, wl.alpha, sigma, tau, theta, p, synth.gate_sequence(N, wl.gate_seed, e))

    for e in range(args.warmup):
        epoch(e)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} epochs done")

    # timed region: exactly K epochs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(args.steps):
        epoch(args.warmup + e)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    log(f"timed {args.steps} epochs: {ms_per_step:.3f} ms/epoch")

    # the same epochs again with every kernel bracketed by HIP events
    h.profile(True)
    h.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(args.steps):
        epoch(args.warmup + args.steps + e)
    torch.cuda.synchronize()
    prof_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kstats = h.profile_read()
    h.profile(False)
    log("kernels: " + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f} us x{v[1]}" for k, v in kstats.items() if v[1]))

    # A_i + A_i^* pairs, cycling over the gates
    xs = xg.clone()
    s = h.new_sino()
    b = h.new_image()
    for i in range(N):
        h.apply_Ai(i, xs, s)
        h.apply_Ai_adjoint(i, s, b)
    torch.cuda.synchronize()
    runs = []
    for _ in range(5):   # median of 5 runs of `pairs` pairs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.pairs):
            i = k % N
            h.apply_Ai(i, xs, s)
            h.apply_Ai_adjoint(i, s, b)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0) / args.pairs)
    pair_s = float(np.median(runs))
    log(f"pairs: {1e6 * pair_s:.1f} us per A_i + A_i^* pair (median of 5 runs of {args.pairs})")

    # the same epochs through the batched path with one slice: the epoch's
    # launch sequence captured once as a HIP graph and replayed, and plain
    from paper_2410_10503_amd import BatchHandle
    bh = BatchHandle(n, na, nd, [N], motion, dtype=torch.float32, device=dev)
    bh.set_variant(variant["fwd"], variant["adj_px"], variant["adj_shares"])
    db = torch.stack(d)
    graph_eps = {}
    for use_graph in (True, False):
        stb = bh.zero_batch_state()
        run = lambda e: bh.batch_spdhg_epoch(stb, db, [wl.alpha], sigma, [tau], [theta], p,  # noqa: E731
                                             [int(g) for g in synth.gate_sequence(N, wl.gate_seed, e)],
                                             use_graph=use_graph)
        for e in range(args.warmup):
            run(e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(args.steps):
            run(args.warmup + e)
        torch.cuda.synchronize()
        graph_eps["graph" if use_graph else "plain"] = args.steps / (time.perf_counter() - t0)
    bh.close()
    del db
    log(f"one-slice batched path: {graph_eps}")

    # roofline of the dominant kernel (per launch)
    nnz = joseph_nnz(n, na, nd)
    img_b, sino_b = 4 * n * n, 4 * na * nd
    work = {  # algorithmic FLOPs and HBM bytes of one launch of each kernel class in the epoch
        "project": (2.0 * nnz, img_b + 4 * sino_b),          # image in; y, d in; y, dy out
        "backproject": (2.0 * nnz, sino_b + img_b),           # dy in, image out
        "warp": (8.0 * n * n, img_b + 2 * img_b + (2 * img_b if wl.motion == "field" else 0)),
        "twarp": (2.0 * 9 * 4 * n * n, img_b * (1 + 5) + (2 * img_b if wl.motion == "field" else 0)),
    }
    dom = max(work, key=lambda k: kstats[k][0])
    tot_ms, cnt = kstats[dom]
    avg_s = tot_ms / 1e3 / max(cnt, 1)
    flops, bytes_ = work[dom]
    if dom in ("project", "backproject"):
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    if roof["bound"] == "alu":
        # the library is built without packed FP32 (one FMA per lane per cycle)
        roof["peak_without_packed_fp32"] = PEAK_FP32_TFLOPS / 2
        roof["frac_without_packed_fp32"] = roof["achieved"] / (PEAK_FP32_TFLOPS / 2)
    roof["traffic"] = measured_traffic(dom, variant)
    roof["kernel"] = dom
    if roof["bound"] == "alu":
        # what binds the class's main kernel: the fraction of the SIMD cycles
        # that issue a VALU instruction (SQ counters of the committed summary)
        vi = measured_valu_issue(dom, variant)
        if vi is not None:
            roof["valu_issue_frac"], roof["valu_insts_per_launch"], roof["valu_kernel"] = vi
    roof["avg_launch_us"] = avg_s * 1e6
    roof["hbm_gbs_algorithmic"] = bytes_ / avg_s / 1e9
    roof["nnz_per_launch"] = nnz
    if dom in ("project", "backproject"):
        roof["weights_per_s"] = nnz / avg_s   # interpolation weights applied per second
        # on-chip reads: the LDS-staged projector kernels read 8 bytes (two
        # floats) per sample, a ray on a line (about nnz / 2 of them) or a
        # pixel at an angle (n^2 n_a), against the LDS read rate measured on
        # the MI355X with 16-byte reads at conflict-free addresses
        samples = nnz / 2.0 if dom == "project" else float(n) * n * na
        roof["lds_read_tbs"] = 8.0 * samples / avg_s / 1e12
        roofs = measured_roofs()  # probe rates of the committed summary
        if roofs:
            roof["lds_read_roof_tbs"] = roofs["lds_read_tbs"]
            roof["lds_frac"] = roof["lds_read_tbs"] / roofs["lds_read_tbs"]
            roof["copy_gbs_measured"] = roofs["copy_gbs"]
            roof["roofs_source"] = os.path.relpath(ROOFS_SUMMARY, ROOT)
    if roof["traffic"]:
        roof["hbm_gbs_measured"] = roof["traffic"] / avg_s / 1e9
        roof["hbm_frac_measured"] = roof["hbm_gbs_measured"] / PEAK_HBM_GBS
    # the pair's HBM bandwidth against half the copy rate: the gather kernels
    # are bound on chip (VALU issue, LDS and L2 latency), so this target of the
    # hot path is not met by design; the fractions above say which roof binds
    roof["hbm_frac_algorithmic"] = roof["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
    roof["pair_hbm_half_of_copy_met"] = bool(
        roof.get("copy_gbs_measured") and roof["hbm_gbs_algorithmic"] >= 0.5 * roof["copy_gbs_measured"])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "SPDHG epochs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded chest-like phantom, displacement fields, Gaussian noise)",
        "config": {"workload": wl.name, "n": n, "n_angles": na, "n_det": nd, "gates": N, "motion": wl.motion,
                   "alpha": wl.alpha},
        "pairs_per_s": 1.0 / pair_s,
        "us_per_pair": pair_s * 1e6,
        "ms_per_step_with_kernel_events": prof_ms,
        "kernels_us_per_launch": {k: (v[0] * 1e3 / v[1] if v[1] else None) for k, v in kstats.items()},
        "projector_variant": variant,
        "epochs_per_s_one_slice_batched": graph_eps,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        bcopy = torch.empty_like(a)
        torch.cuda.synchronize()
        bcopy.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 4
        del a, bcopy
    if not args.no_subsets:
        for i, M in enumerate(int(m) for m in args.subsets_m.split(",")):
            key = "subsets" if i == 0 else f"subsets_m{M}"
            log(f"gates x {M} angle subsets ...")
            out[key] = subsets_measurement(h, d, wl, norms, v0, value, variant, M=M)
            log(f"{key}: {out[key]}")
    if not args.no_pdhg:
        log("PDHG vs SPDHG on the 512^2 rigid workload ...")
        out["pdhg_vs_spdhg"] = pdhg_spdhg_measurement()
        log(f"pdhg_vs_spdhg: {out['pdhg_vs_spdhg']}")
    if not args.no_batch:
        log("batched workload: 64 slices of 256^2 ...")
        out["batched"] = batched_measurement(max(2, args.steps // 3))
        log(f"batched: {out['batched']}")
    if not args.no_autograd:
        log("differentiation through 10 unrolled iterations ...")
        out["autograd"] = autograd_measurement()
        log(f"autograd: {out['autograd']}")
    if not args.no_registration:
        log("rigid registration of 16 gates ...")
        out["registration"] = registration_measurement()
        log(f"registration: {out['registration']}")
    out["cpu_baseline"] = cpu_leg
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
