"""GPU parity of the operators (warp, projector, their transposes, A_i and
A_i^*) against the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_common import F32_OP, F64_OP, Problem, dev, f32, host, need_gpu, rel, rel_max
import synth
from oracle import projector, warp

pytestmark = pytest.mark.gpu

DT = [(torch.float32, F32_OP), (torch.float64, F64_OP)]
# (n, n_angles, n_det): several detector tiles with a ragged tail, the 45/135
# degree ties present (n_angles divisible by 4), odd and even sizes
GEOMS = [(64, 96, 92), (75, 40, 300), (128, 120, 182)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("dtype,bar", DT)
@pytest.mark.parametrize("geom", GEOMS)
def test_project_and_backproject(dtype, bar, geom):
    n, na, nd = geom
    P = Problem(n, na, nd, 1, "identity")
    h = P.handle(dtype)
    x = f32(synth.ellipse_phantom(n, 3)) + f32(synth.random_image(n, 4)) * 0.1
    y = f32(synth.random_sinograms(1, na, nd, 5)[0])
    s = host(h.project(dev(x, dtype)))
    b = host(h.backproject(dev(y, dtype)))
    assert rel(s, projector.forward(x, na, nd)) < bar
    assert rel(b, projector.adjoint(y, n)) < bar


# (forward, adjoint pixels per thread, adjoint angle shares)
VARIANTS = [(0, 0, 1), (1, 0, 1), (1, 1, 1), (1, 2, 2), (1, 4, 1), (1, 4, 4), (0, 4, 3), (2, 4, 4), (2, 2, 1),
            (3, 4, 4), (3, 1, 2), (3, 4, 8), (2, 2, 7), (3, 8, 4), (0, 8, 1),
            # quarter-turn adjoint (falls back to the tiled one on odd sizes)
            (3, -4, 6), (3, -2, 1), (3, -8, 8), (0, -4, 3), (2, -2, 5),
            # quarter-turn forward (unavailable on odd sizes)
            (4, -4, 8), (4, 4, 4), (4, 8, 6), (4, -2, 16), (4, -16, 8), (4, -32, 16), (3, -32, 3),
            # eight-plane forward (n even, n_angles a multiple of 4)
            (5, -4, 8), (5, 4, 4), (5, 8, 6), (5, -2, 16)]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("geom", [(64, 96, 92), (75, 40, 300), (200, 90, 290), (33, 16, 48), (96, 720, 140),
                                  (100, 60, 151)])
def test_projector_variants(variant, geom):
    from paper_2410_10503_amd import McrError
    n, na, nd = geom
    P = Problem(n, na, nd, 2, "rigid")
    h = P.handle(torch.float32)
    try:
        h.set_variant(*variant)
    except McrError as e:
        assert "do not fit" in str(e)
        h.set_variant(0, variant[1], variant[2])
    x = f32(synth.ellipse_phantom(n, 3)) + f32(synth.random_image(n, 4)) * 0.1
    y = f32(synth.random_sinograms(1, na, nd, 5)[0])
    assert rel(host(h.project(dev(x, torch.float32))), projector.forward(x, na, nd)) < F32_OP
    assert rel(host(h.backproject(dev(y, torch.float32))), projector.adjoint(y, n)) < F32_OP
    assert rel(host(h.apply_Ai(1, dev(x, torch.float32))), P.ops.A(1, x)) < F32_OP
    assert rel(host(h.apply_Ai_adjoint(1, dev(y, torch.float32))), P.ops.At(1, y)) < F32_OP


def test_autotune_keeps_parity():
    P = Problem(128, 120, 182, 3, "field")
    h = P.handle(torch.float32)
    choice = h.autotune(1)
    assert choice["fwd"] in (0, 1, 2, 3, 4, 5) and choice["adj_px"] in (0, 1, 2, 4, 8, -2, -4, -8, -16, -32)
    assert 1 <= choice["adj_shares"] <= 16
    assert h.autotune(3) is not None
    x = f32(synth.ellipse_phantom(128, 1))
    y = f32(synth.random_sinograms(1, 120, 182, 2)[0])
    for i in range(3):
        assert rel(host(h.apply_Ai(i, dev(x, torch.float32))), P.ops.A(i, x)) < F32_OP
        assert rel(host(h.apply_Ai_adjoint(i, dev(y, torch.float32))), P.ops.At(i, y)) < F32_OP


@pytest.mark.parametrize("dtype,bar", DT)
@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_warp_and_transpose(dtype, bar, kind):
    n = 96
    P = Problem(n, 8, 140, 4, kind, field_scale=2.0)
    h = P.handle(dtype)
    x = f32(synth.ellipse_phantom(n, 7))
    b = f32(synth.random_image(n, 8))
    for i in range(P.N):
        pos = P.ops.pos[i]
        w = host(h.warp(i, dev(x, dtype)))
        wt = host(h.warp_adjoint(i, dev(b, dtype)))
        if P.kind == "field" and i == 0:
            np.testing.assert_array_equal(w, x)        # gate 0 of the field model is the identity
        assert rel(w, warp.warp(x, *pos)) < bar
        assert rel(wt, warp.warp_adjoint(b, *pos)) < bar


@pytest.mark.parametrize("dtype,bar", DT)
@pytest.mark.parametrize("kind", ["identity", "rigid", "field"])
def test_apply_Ai_pair(dtype, bar, kind):
    n, na, nd = 80, 60, 116
    P = Problem(n, na, nd, 3, kind, field_scale=1.5)
    h = P.handle(dtype)
    x = f32(synth.ellipse_phantom(n, 1))
    y = f32(synth.random_sinograms(1, na, nd, 2)[0])
    for i in range(P.N):
        assert rel(host(h.apply_Ai(i, dev(x, dtype))), P.ops.A(i, x)) < bar
        assert rel(host(h.apply_Ai_adjoint(i, dev(y, dtype))), P.ops.At(i, y)) < bar


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 2e-6), (torch.float64, 1e-13)])
@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_dot_product(dtype, tol, kind):
    n, na, nd = 128, 120, 182
    P = Problem(n, na, nd, 2, kind)
    h = P.handle(dtype)
    x = dev(f32(synth.random_image(n, 11)), dtype)
    y = dev(f32(synth.random_sinograms(1, na, nd, 12)[0]), dtype)
    for i in range(P.N):
        ax = h.apply_Ai(i, x)
        aty = h.apply_Ai_adjoint(i, y)
        lhs = float(torch.sum(ax.double() * y.double()))
        rhs = float(torch.sum(x.double() * aty.double()))
        assert abs(lhs - rhs) <= tol * float(ax.double().norm() * y.double().norm())


@pytest.mark.parametrize("kind", ["rigid", "field"])
def test_matrix_16x16(kind):
    # assemble the FP32 GPU forward and adjoint matrices column by column; the
    # adjoint's entries are the forward's (the same floating-point weights)
    n, na, nd = 16, 12, 24
    P = Problem(n, na, nd, 1, kind, max_rot=20.0, max_shift=2.5, field_scale=0.4)
    h = P.handle(torch.float32)
    e = torch.zeros(n * n, device="cuda")
    mf = np.zeros((na * nd, n * n))
    for q in range(n * n):
        e.zero_()
        e[q] = 1
        mf[:, q] = host(h.apply_Ai(0, e.view(n, n))).ravel()
    es = torch.zeros(na * nd, device="cuda")
    ma = np.zeros((n * n, na * nd))
    for q in range(na * nd):
        es.zero_()
        es[q] = 1
        ma[:, q] = host(h.apply_Ai_adjoint(0, es.view(na, nd))).ravel()
    scale = np.abs(mf).max()
    assert np.abs(ma - mf.T).max() <= 1e-6 * scale
    # both against the oracle's dense matrix of A D_0
    ident = np.eye(n * n)
    mo = np.stack([P.ops.A(0, ident[q].reshape(n, n)).ravel() for q in range(n * n)], axis=1)
    assert np.abs(mf - mo).max() <= 2e-6 * scale


def test_determinism():
    n, na, nd = 128, 120, 182
    P = Problem(n, na, nd, 2, "field")
    h = P.handle(torch.float32)
    x = dev(f32(synth.random_image(n, 1)), torch.float32)
    y = dev(f32(synth.random_sinograms(1, na, nd, 2)[0]), torch.float32)
    a1, a2 = h.apply_Ai(1, x), h.apply_Ai(1, x)
    b1, b2 = h.apply_Ai_adjoint(1, y), h.apply_Ai_adjoint(1, y)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


@pytest.mark.parametrize("variant", ["autotune", (4, -4, 12), (5, -4, 12)])
def test_full_size_field_gate(variant):
    # 512^2, 720 angles x 730 bins, the headline chest phantom and one
    # non-rigid gate, in the configuration the benchmark times (the variants
    # the autotuner keeps) and with each quarter-turn forward
    P = Problem(512, 720, 730, 16, "field", phantom="chest")
    h = P.handle(torch.float32)
    if variant == "autotune":
        h.autotune(1)
    else:
        h.set_variant(*variant)
    i = 11
    x = P.x_true
    s = host(h.apply_Ai(i, dev(x, torch.float32)))
    s_ref = P.ops.A(i, x)
    assert rel(s, s_ref) < F32_OP
    # no single ray off by more than the bar, relative to the largest ray sum
    assert rel_max(s, s_ref) < F32_OP
    y = f32(synth.random_sinograms(1, 720, 730, 9)[0])
    b = host(h.apply_Ai_adjoint(i, dev(y, torch.float32)))
    b_ref = P.ops.At(i, y)
    assert rel(b, b_ref) < F32_OP
    assert rel_max(b, b_ref) < F32_OP
    assert h.info()["window_radius"] == 1


def test_full_size_rigid_samples():
    # all 16 rigid gates at 512^2: sampled rays of A_i x and sampled pixels of
    # D_i^T b against the oracle, one by one
    P = Problem(512, 720, 730, 16, "rigid")
    h = P.handle(torch.float32)
    h.autotune(1)
    x = P.x_true
    xd = dev(x, torch.float32)
    rng = np.random.default_rng(0)
    b = f32(synth.random_image(512, 3))
    for i in range(16):
        s = host(h.apply_Ai(i, xd))
        w = warp.warp(x, *P.ops.pos[i])
        for _ in range(6):
            k, j = int(rng.integers(720)), int(rng.integers(730))
            ref = projector.ray_sum(w, 720, 730, k, j)
            assert abs(s[k, j] - ref) <= 1e-5 * max(1.0, abs(ref)) + 1e-5 * np.abs(s).max()
        wt = host(h.warp_adjoint(i, dev(b, torch.float32)))
        assert rel(wt, warp.warp_adjoint(b, *P.ops.pos[i])) < F32_OP


def test_argument_errors():
    from paper_2410_10503_amd import McrError
    P = Problem(32, 20, 48, 2, "rigid")
    h = P.handle(torch.float32)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(McrError, match="gate 2 out of range"):
        h.apply_Ai(2, x)
    st = h.zero_state()
    d = [torch.zeros(20, 48, device="cuda") for _ in range(2)]
    with pytest.raises(McrError, match="p\\[1\\]"):
        h.spdhg_iterate(st, d, 1.0, [1.0, 1.0], 1.0, 0.5, [0.5, 1.5], [0])
    with pytest.raises(McrError, match="sigma\\[0\\]"):
        h.spdhg_iterate(st, d, 1.0, [float("nan"), 1.0], 1.0, 0.5, [0.5, 0.5], [0])
    with pytest.raises(McrError, match="alpha"):
        h.pdhg_epoch(st, d, -1.0, [1.0, 1.0], 1.0, 0.5)


@pytest.mark.parametrize("geom", [(1024, 1440, 1450), (300, 97, 120), (257, 512, 700)])
def test_large_and_odd_geometries_sampled(geom):
    # a 1024^2 image with 1440 angles (four times the headline's pixels), a
    # detector narrower than the image with an odd angle count (no 45/135
    # degree ties), and a wide detector on an odd image size: sampled rays of
    # A x and sampled pixels of A^T y against the oracle, one by one, for every
    # float32 forward variant that fits and the default adjoint
    from paper_2410_10503_amd import McrError
    n, na, nd = geom
    P = Problem(n, na, nd, 1, "identity")
    h = P.handle(torch.float32)
    x = f32(synth.ellipse_phantom(n, 3))
    y = f32(synth.random_sinograms(1, na, nd, 5)[0])
    rng = np.random.default_rng(n)
    rays = [(int(rng.integers(na)), int(rng.integers(nd))) for _ in range(16)]
    pix = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(2)]
    refs = [projector.ray_sum(x, na, nd, k, j) for k, j in rays]
    prefs = [projector.backproject_pixel(y, n, r, c) for r, c in pix]
    for adj in ((8, 6), (-4, 6)):
        h.set_variant(0, *adj)
        b = host(h.backproject(dev(y, torch.float32)))
        for (r, c), ref in zip(pix, prefs):
            assert abs(b[r, c] - ref) <= 1e-5 * np.abs(b).max(), (adj, r, c, b[r, c], ref)
    for fwd in (0, 1, 2, 3, 4, 5):
        try:
            h.set_variant(fwd, 8, 6)
        except McrError as e:
            assert "do not fit" in str(e)
            continue
        s = host(h.project(dev(x, torch.float32)))
        for (k, j), ref in zip(rays, refs):
            assert abs(s[k, j] - ref) <= 1e-5 * np.abs(s).max(), (fwd, k, j, s[k, j], ref)


@pytest.mark.parametrize("geom", [(1, 1, 1), (2, 3, 1), (3, 1, 5), (5, 4, 2), (2, 8, 7), (7, 2, 40), (6, 4, 41),
                                  (64, 8, 9)])
def test_degenerate_geometries(geom):
    # one pixel, one angle, one detector bin, and detectors far wider or
    # narrower than the image: every variant against the oracle
    from paper_2410_10503_amd import McrError
    n, na, nd = geom
    x = np.arange(n * n, dtype=np.float64).reshape(n, n) + 1.0
    y = np.arange(na * nd, dtype=np.float64).reshape(na, nd) + 0.5
    s_ref, b_ref = projector.forward(x, na, nd), projector.adjoint(y, n)
    for dtype, bar in DT:
        P = Problem(n, na, nd, 1, "identity")
        h = P.handle(dtype)
        variants = [None] if dtype == torch.float64 else [(0, 0, 1), (1, 1, 1), (2, 2, 2), (3, 4, 1), (3, 8, 3),
                                                          (3, -4, 1), (3, -2, 3), (3, -8, 8), (4, -4, 1),
                                                          (4, 8, 2), (4, -16, 1), (4, -32, 5), (5, -4, 1),
                                                          (5, 8, 2)]
        for v in variants:
            if v is not None:
                try:
                    h.set_variant(*v)
                except McrError as e:
                    assert "do not fit" in str(e)
                    continue
            s = host(h.project(dev(x, dtype)))
            b = host(h.backproject(dev(y, dtype)))
            assert np.abs(s - s_ref).max() <= bar * max(np.abs(s_ref).max(), 1.0), (v, s, s_ref)
            assert np.abs(b - b_ref).max() <= bar * max(np.abs(b_ref).max(), 1.0), (v, b, b_ref)


def test_maximum_image_size_sampled():
    # n = 4096, the largest image the library accepts (few angles keep it
    # cheap): sampled rays of A x and one pixel of A^T y against the oracle
    n, na, nd = 4096, 48, 5800
    P = Problem(n, na, nd, 1, "identity")
    h = P.handle(torch.float32)
    x = f32(synth.ellipse_phantom(n, 3))
    y = f32(synth.random_sinograms(1, na, nd, 5)[0])
    s = host(h.project(dev(x, torch.float32)))
    rng = np.random.default_rng(4096)
    for _ in range(8):
        k, j = int(rng.integers(na)), int(rng.integers(nd))
        ref = projector.ray_sum(x, na, nd, k, j)
        assert abs(s[k, j] - ref) <= 1e-5 * np.abs(s).max(), (k, j, s[k, j], ref)
    b = host(h.backproject(dev(y, torch.float32)))
    ref = projector.backproject_pixel(y, n, 1000, 2000)
    assert abs(b[1000, 2000] - ref) <= 1e-5 * np.abs(b).max()
