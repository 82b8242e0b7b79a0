"""GPU parity of the rigid registration (mcr_register_rigid) against the FP64
oracle (oracle/registration.py, the same reading of the preliminary step of
Section I), and recovery of known rigid motions, through the C ABI."""
import numpy as np
import pytest
import torch
from scipy import ndimage

from gpu_common import Problem, dev, f32, need_gpu
import synth
from oracle import registration as oreg, warp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _ref(n, seed=3, blur=1.5):
    # a smooth reference (blurred ellipses), rounded to float32 for both sides
    return f32(ndimage.gaussian_filter(synth.ellipse_phantom(n, seed).astype(np.float64), blur * n / 64))


def _target(ref, theta):
    return f32(warp.warp(ref, *warp.rigid_positions(ref.shape[0], *theta)))


def _px(theta, n):
    return np.asarray(theta, float) * np.array([(n - 1) / 2.0, 1.0, 1.0])


@pytest.mark.parametrize("theta", [(0.05, 1.7, -2.3), (-0.087, 3.9, 0.6)])
def test_fp64_registration_matches_oracle(theta):
    n = 64
    P = Problem(n, 40, 92, 2, "rigid")
    ref = _ref(n)
    tgt = _target(ref, theta)
    th_o, E_o, k_o = oreg.register_rigid(ref, tgt, max_iter=300, tol=1e-9)
    h = P.handle(torch.float64)
    th, E, k = h.register_rigid(1, dev(ref, torch.float64), dev(tgt, torch.float64), max_iter=300, tol=1e-9)
    # the same iteration on the same data: the same path up to rounding
    assert k == k_o
    assert np.abs(_px(th, n) - _px(th_o, n)).max() < 1e-9
    assert np.abs(_px(th, n) - _px(theta, n)).max() < 1e-6
    assert abs(E - E_o) <= 1e-12 * float(np.sum(tgt ** 2))
    # the gate's motion is the result: D ref reproduces the target
    w = h.warp(1, dev(ref, torch.float64)).cpu().numpy()
    assert np.abs(w - tgt).max() < 1e-6 * np.abs(tgt).max()


def test_energy_at_start_matches_oracle():
    n = 64
    P = Problem(n, 40, 92, 2, "rigid")
    ref, tgt = _ref(n), _target(_ref(n, seed=5), (0.02, 0.5, -0.5))
    start = (0.03, 1.2, -0.7)
    E_o, _ = oreg.energy_and_grad(ref, tgt, start)
    for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        h = P.handle(dtype)
        th, E, k = h.register_rigid(0, dev(ref, dtype), dev(tgt, dtype), params=start, max_iter=0)
        assert k == 0 and th == start
        assert abs(E - E_o) <= bar * E_o


def test_full_size_fp32_recovers_sixteen_gates():
    # 512^2, the 16 rigid gates of the 512^2 rigid workload (rotations up to
    # 8 degrees, shifts up to 10 px): each gate's image is the reference warped
    # by its motion (oracle warp); registration from zero in float32
    n = 512
    P = Problem(n, 720, 730, 16, "rigid")
    h = P.handle(torch.float32)
    ref = _ref(n)
    rd = dev(ref, torch.float32)
    for i in range(16):
        tgt = _target(ref, P.params[i])
        th, E, k = h.register_rigid(i, rd, dev(tgt, torch.float32), max_iter=300, tol=1e-5)
        err = np.abs(_px(th, n) - _px(P.params[i], n)).max()
        assert err < 2e-3, (i, th, P.params[i], err, k)


def test_registration_arguments():
    from paper_2410_10503_amd import McrError
    P = Problem(32, 20, 48, 2, "field")
    h = P.handle(torch.float32)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(McrError, match="not rigid"):
        h.register_rigid(0, x, x)
    R = Problem(32, 20, 48, 2, "rigid")
    hr = R.handle(torch.float32)
    with pytest.raises(McrError, match="params"):
        hr.register_rigid(0, x, x, params=(float("nan"), 0.0, 0.0))
    with pytest.raises(McrError, match="max_iter"):
        hr.register_rigid(0, x, x, max_iter=-1)
    th, E, k = hr.register_rigid(1, x, x)  # zero images: zero gradient, no step
    assert k == 0 and E == 0.0


def _affine_target(ref, theta):
    return f32(warp.warp(ref, *warp.field_positions(oreg.affine_field(ref.shape[0], theta))))


def _apx(theta, n):
    return np.asarray(theta, float) * np.array([(n - 1) / 2.0] * 4 + [1.0, 1.0])


def _rot_affine(phi, tx, ty):
    return (np.cos(phi) - 1.0, -np.sin(phi), np.sin(phi), np.cos(phi) - 1.0, tx, ty)


@pytest.mark.parametrize("theta", [(0.0, 0.0, 0.0, 0.06, 0.5, -1.0), _rot_affine(0.05, 1.7, -2.3)])
def test_fp64_affine_registration_matches_oracle(theta):
    n = 64
    P = Problem(n, 40, 92, 2, "field")
    ref = _ref(n)
    tgt = _affine_target(ref, theta)
    th_o, E_o, k_o = oreg.register_affine(ref, tgt, max_iter=500, tol=1e-9)
    h = P.handle(torch.float64)
    th, E, k = h.register_affine(1, dev(ref, torch.float64), dev(tgt, torch.float64), max_iter=500, tol=1e-9)
    assert k == k_o
    assert np.abs(_apx(th, n) - _apx(th_o, n)).max() < 1e-9
    assert np.abs(_apx(th, n) - _apx(theta, n)).max() < 1e-5
    assert abs(E - E_o) <= 1e-12 * float(np.sum(tgt ** 2))


def test_affine_energy_at_start_and_installed_field():
    n = 64
    P = Problem(n, 40, 92, 2, "field")
    ref, tgt = _ref(n), _affine_target(_ref(n, seed=5), (0.01, 0.0, 0.0, 0.04, 0.3, -0.2))
    start = (0.004, -0.01, 0.02, 0.03, 0.6, 0.2)
    E_o, _ = oreg.energy_and_grad_affine(ref, tgt, start)
    b = f32(synth.random_image(n, 8))
    for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        h = P.handle(dtype)
        th, E, k = h.register_affine(0, dev(ref, dtype), dev(tgt, dtype), params=start, max_iter=0)
        assert k == 0 and th == start
        assert abs(E - E_o) <= bar * E_o
        # the gate now carries the start map: its warp and transposed warp
        # against the oracle's with the same (float32) field
        pos = warp.field_positions(oreg.affine_field(n, start))
        assert np.abs(h.warp(0, dev(ref, dtype)).cpu().numpy() - warp.warp(ref, *pos)).max() <= 10 * bar
        wt = h.warp_adjoint(0, dev(b, dtype)).cpu().numpy()
        ref_wt = warp.warp_adjoint(b, *pos)
        assert np.linalg.norm(wt - ref_wt) <= 10 * bar * np.linalg.norm(ref_wt)


def test_full_size_fp32_recovers_ten_dilatations():
    # 512^2, 10 field gates with the chest experiment's motion kind: vertical
    # linear dilatations growing with the gate phase (up to 8 px at the edge)
    # plus small shifts; each registered from zero in float32
    n = 512
    P = Problem(n, 720, 730, 10, "field")
    h = P.handle(torch.float32)
    ref = _ref(n)
    rd = dev(ref, torch.float32)
    for i in range(10):
        q = i / 9.0
        theta = (0.0, 0.0, 0.0, 8.0 * q / 255.5, 0.5 * q, -0.7 * q)
        tgt = _affine_target(ref, theta)
        th, E, k = h.register_affine(i, rd, dev(tgt, torch.float32), max_iter=500, tol=1e-5)
        err = np.abs(_apx(th, n) - _apx(theta, n)).max()
        assert err < 2e-3, (i, th, theta, err, k)


def test_affine_registration_arguments():
    from paper_2410_10503_amd import McrError
    R = Problem(32, 20, 48, 2, "rigid")
    hr = R.handle(torch.float32)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(McrError, match="not a field gate"):
        hr.register_affine(0, x, x)
    P = Problem(32, 20, 48, 2, "field")
    h = P.handle(torch.float32)
    with pytest.raises(McrError, match="params"):
        h.register_affine(0, x, x, params=(0.0, float("inf"), 0.0, 0.0, 0.0, 0.0))
    th, E, k = h.register_affine(1, x, x)
    assert k == 0 and E == 0.0


# -- dense displacement fields (mcr_register_field) ---------------------------

def _bump_field(n, ax, ay, sigma):
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    b = np.exp(-((xx - c) ** 2 + (yy - c) ** 2) / (2 * sigma * sigma))
    return f32(np.stack([ax * b, ay * b]))


def _field_target(ref, u):
    return f32(warp.warp(ref, *warp.field_positions(u)))


def test_fp64_field_registration_matches_oracle():
    n = 48
    P = Problem(n, 40, 70, 2, "field")
    ref = _ref(n)
    tgt = _field_target(ref, _bump_field(n, 1.2, -0.8, 10.0))
    u_o, E_o, k_o = oreg.register_field(ref, tgt, lam=0.01, max_iter=60, tol=1e-4)
    h = P.handle(torch.float64)
    u, E, k = h.register_field(1, dev(ref, torch.float64), dev(tgt, torch.float64), lam=0.01, max_iter=60,
                               tol=1e-4)
    # the same iteration on the same data: the same path up to rounding
    print("fp64 field registration: steps", k, k_o, "E", E, E_o)
    assert k == k_o
    assert np.abs(u.cpu().numpy() - f32(u_o)).max() < 1e-5
    assert abs(E - E_o) <= 1e-9 * E_o


def test_field_energy_at_start_and_installed_field():
    n = 48
    P = Problem(n, 40, 70, 2, "field")
    ref, tgt = _ref(n), _field_target(_ref(n, seed=5), _bump_field(n, 0.7, 0.4, 8.0))
    rng = np.random.default_rng(3)
    start = f32(_bump_field(n, -0.5, 0.9, 12.0) + rng.uniform(-0.2, 0.2, size=(2, n, n)))
    lam = 0.2
    E_o, _ = oreg.energy_and_grad_field(ref, tgt, start, lam)
    b = f32(synth.random_image(n, 8))
    pos = warp.field_positions(start)
    for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        h = P.handle(dtype)
        f = torch.from_numpy(start.astype(np.float32)).cuda()
        u, E, k = h.register_field(0, dev(ref, dtype), dev(tgt, dtype), field=f, lam=lam, max_iter=0)
        assert k == 0 and torch.equal(u.cpu(), torch.from_numpy(start.astype(np.float32)))
        assert abs(E - E_o) <= bar * E_o, (dtype, E, E_o)
        # the gate now carries the start field: warp and transposed warp
        assert np.abs(h.warp(0, dev(ref, dtype)).cpu().numpy() - warp.warp(ref, *pos)).max() <= 10 * bar
        wt = h.warp_adjoint(0, dev(b, dtype)).cpu().numpy()
        ref_wt = warp.warp_adjoint(b, *pos)
        assert np.linalg.norm(wt - ref_wt) <= 10 * bar * np.linalg.norm(ref_wt)


def test_fp32_field_registration_tracks_oracle():
    n = 64
    P = Problem(n, 40, 92, 2, "field")
    ref = _ref(n)
    ustar = _bump_field(n, 1.5, -1.0, 12.0)
    tgt = _field_target(ref, ustar)
    h = P.handle(torch.float32)
    rd, td = dev(ref, torch.float32), dev(tgt, torch.float32)
    # the first step (the normalised gradient, halved by the same Armijo
    # tests): float32 rounding of the gradient only
    u1_o, E1_o, _ = oreg.register_field(ref, tgt, lam=0.01, max_iter=1, tol=1e-4)
    u1, E1, k1 = h.register_field(1, rd, td, lam=0.01, max_iter=1, tol=1e-4)
    assert k1 == 1
    assert np.abs(u1.cpu().numpy() - u1_o).max() < 1e-4
    assert abs(E1 - E1_o) <= 1e-4 * E1_o
    # 40 steps: the Barzilai-Borwein lengths amplify the rounding, so the
    # paths part; both descend alike (energy, distance to the true field)
    u_o, E_o, k_o = oreg.register_field(ref, tgt, lam=0.01, max_iter=40, tol=1e-4)
    u, E, k = h.register_field(1, rd, td, field=torch.zeros(2, n, n, device="cuda"), lam=0.01, max_iter=40,
                               tol=1e-4)
    gm = np.hypot(*np.gradient(ref))
    m = gm > 0.1 * gm.max()
    err = np.sqrt(np.mean(np.sum((u.cpu().numpy() - ustar) ** 2, axis=0)[m]))
    err_o = np.sqrt(np.mean(np.sum((u_o - ustar) ** 2, axis=0)[m]))
    print("fp32 field registration: steps", k, k_o, "E", E, E_o, "rms error", err, err_o)
    assert abs(E - E_o) <= 5e-2 * E_o
    assert err <= 1.2 * err_o + 0.01


def test_full_size_fp32_affine_then_dense():
    # 512^2 (the headline image size): a vertical dilatation of up to 4 px at
    # the edges plus a smooth bump of up to 2 px; the affine registration
    # takes the dilatation, the dense registration started from its field
    # then lowers the misfit and the distance to the true field further (a
    # single-level descent: slow on this smooth reference, so 300 steps give
    # a partial refinement; the FP64 oracle on the same problem reaches 0.68
    # of the affine misfit and 0.82 of its field error)
    n = 512
    P = Problem(n, 720, 730, 2, "field")
    h = P.handle(torch.float32)
    ref = _ref(n)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    b = np.exp(-((xx - c - 0.1 * n) ** 2 + (yy - c) ** 2) / (2 * (0.12 * n) ** 2))
    ustar = f32(np.stack([2.0 * b, -1.4 * b + 4.0 * (yy - c) / c]))
    tgt = _field_target(ref, ustar)
    rd, td = dev(ref, torch.float32), dev(tgt, torch.float32)
    th, Ea, ka = h.register_affine(1, rd, td, max_iter=300, tol=1e-5)
    ua = f32(np.stack([(th[0] * (xx - c) + th[1] * (yy - c)) + th[4], (th[2] * (xx - c) + th[3] * (yy - c)) + th[5]]))
    lam = 0.1
    E_aff, _ = oreg.energy_and_grad_field(ref, tgt, ua, lam)
    u, E, k = h.register_field(1, rd, td, field=torch.from_numpy(ua.astype(np.float32)).cuda(), lam=lam,
                               max_iter=300, tol=1e-3)
    gm = np.hypot(*np.gradient(ref))
    m = gm > 0.1 * gm.max()
    rms = lambda v: np.sqrt(np.mean(np.sum(v ** 2, axis=0)[m]))  # noqa: E731
    err_aff, err = rms(ua - ustar), rms(u.cpu().numpy() - ustar)
    print("512^2: affine", ka, "steps; dense", k, "steps, E", E_aff, "->", E, "rms error", err_aff, "->", err)
    assert E <= 0.8 * E_aff
    assert err <= 0.9 * err_aff
    # the gate's field is the result
    w = h.warp(1, rd).cpu().numpy()
    assert np.abs(w - warp.warp(ref, *warp.field_positions(u.cpu().numpy()))).max() < 1e-4


def test_field_registration_arguments():
    from paper_2410_10503_amd import McrError
    R = Problem(32, 20, 48, 2, "rigid")
    hr = R.handle(torch.float32)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(McrError, match="not a field gate"):
        hr.register_field(0, x, x)
    P = Problem(32, 20, 48, 2, "field")
    h = P.handle(torch.float32)
    with pytest.raises(McrError, match="lambda"):
        h.register_field(0, x, x, lam=-1.0)
    u, E, k = h.register_field(1, x, x)
    assert k == 0 and E == 0.0 and not u.any()
    for bad in ((40.0,), (-1.0,), (float("nan"),)):
        with pytest.raises(McrError, match="sigmas"):
            h.register_field(1, x, x, sigmas=bad)
    with pytest.raises(McrError, match="n_levels"):
        h.register_field(1, x, x, sigmas=(1.0,) * 17)
    # a start field that compresses the rows tenfold needs a wider gather
    # window than the transposed warp has: the gate falls back to the identity
    n = 32
    yy = np.mgrid[0:n, 0:n][0].astype(np.float64)
    fold = np.zeros((2, n, n), np.float32)
    fold[1] = -0.9 * (yy - (n - 1) / 2.0)
    img = dev(f32(synth.random_image(n, 2)), torch.float32)
    with pytest.raises(McrError, match="reset to the identity"):
        h.register_field(0, img, img, field=torch.from_numpy(fold).cuda(), max_iter=0)
    assert torch.equal(h.warp(0, img), img)


def test_fp64_scale_space_registration_matches_oracle():
    n = 48
    P = Problem(n, 40, 70, 2, "field")
    ref = _ref(n)
    yy = np.mgrid[0:n, 0:n][0].astype(np.float64)
    ustar = _bump_field(n, 1.0, -0.7, 8.0)
    ustar[1] = f32(ustar[1] + 1.5 * (yy - (n - 1) / 2.0) / ((n - 1) / 2.0))
    tgt = _field_target(ref, ustar)
    sig = (3.0, 1.5, 0.0)
    h = P.handle(torch.float64)
    rd, td = dev(ref, torch.float64), dev(tgt, torch.float64)
    # 8 steps per level: the same path up to rounding
    u_o, E_o, k_o = oreg.register_field(ref, tgt, lam=0.05, max_iter=8, tol=1e-4, sigmas=sig)
    u, E, k = h.register_field(1, rd, td, lam=0.05, max_iter=8, tol=1e-4, sigmas=sig)
    print("fp64 scale-space registration, 8 steps per level: steps", k, k_o, "E", E, E_o)
    assert k == k_o
    assert np.abs(u.cpu().numpy() - f32(u_o)).max() < 1e-4
    assert abs(E - E_o) <= 1e-6 * E_o
    # 40 steps per level: the field is evaluated in float32, so a last-bit
    # difference of the smoothed images (exp, summation order) can move a
    # float32 rounding of the field, which the step lengths then amplify
    # (one level of 40 steps stays within 2e-7 px; across three levels the
    # paths part by up to ~0.02 px): the same energy to 1%
    u_o, E_o, k_o = oreg.register_field(ref, tgt, lam=0.05, max_iter=40, tol=1e-4, sigmas=sig)
    u, E, k = h.register_field(1, rd, td, field=torch.zeros(2, n, n, device="cuda"), lam=0.05, max_iter=40,
                               tol=1e-4, sigmas=sig)
    du = float(np.abs(u.cpu().numpy() - f32(u_o)).max())
    print("fp64 scale-space registration, 40 steps per level: steps", k, k_o, "E", E, E_o, "max du", du)
    assert k == k_o
    assert abs(E - E_o) <= 1e-2 * E_o
    assert du < 0.05


@pytest.mark.parametrize("sigma", [0.8, 2.5, 6.0])
def test_scale_space_energy_at_start(sigma):
    # one level of width sigma, no steps: the energy of the smoothed images
    # at the start field, against the oracle's smoothing and energy
    n = 40
    P = Problem(n, 30, 60, 2, "field")
    ref, tgt = _ref(n), _field_target(_ref(n, seed=5), _bump_field(n, 0.7, 0.4, 8.0))
    start = f32(_bump_field(n, -0.5, 0.9, 10.0))
    E_o, _ = oreg.energy_and_grad_field(oreg.gaussian_smooth(ref, sigma), oreg.gaussian_smooth(tgt, sigma), start,
                                        0.2)
    for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        h = P.handle(dtype)
        f = torch.from_numpy(start.astype(np.float32)).cuda()
        u, E, k = h.register_field(0, dev(ref, dtype), dev(tgt, dtype), field=f, lam=0.2, max_iter=0,
                                   sigmas=(sigma,))
        assert k == 0
        assert abs(E - E_o) <= bar * E_o, (dtype, E, E_o)


def test_full_size_fp32_scale_space_from_zero():
    # 512^2, the same motion as the affine-then-dense case (dilatation up to
    # 4 px + a 2 px bump), registered from zero through a coarse-to-fine
    # schedule (the FP64 oracle on the same problem: misfit to 0.067, field
    # error at edge pixels to 0.75 of the true field's size; the component
    # along an edge is not determined by the data)
    n = 512
    P = Problem(n, 720, 730, 2, "field")
    h = P.handle(torch.float32)
    ref = _ref(n)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    b = np.exp(-((xx - c - 0.1 * n) ** 2 + (yy - c) ** 2) / (2 * (0.12 * n) ** 2))
    ustar = f32(np.stack([2.0 * b, -1.4 * b + 4.0 * (yy - c) / c]))
    tgt = _field_target(ref, ustar)
    lam = 0.1
    E0, _ = oreg.energy_and_grad_field(ref, tgt, np.zeros((2, n, n)), lam)
    u, E, k = h.register_field(1, dev(ref, torch.float32), dev(tgt, torch.float32), lam=lam, max_iter=150,
                               tol=1e-3, sigmas=(8.0, 4.0, 2.0, 1.0, 0.0))
    gm = np.hypot(*np.gradient(ref))
    m = gm > 0.1 * gm.max()
    rms = lambda v: np.sqrt(np.mean(np.sum(v ** 2, axis=0)[m]))  # noqa: E731
    err, err0 = rms(u.cpu().numpy() - ustar), rms(ustar)
    print("512^2 scale-space registration: steps", k, "E", E0, "->", E, "rms error", err0, "->", err)
    assert E < 0.1 * E0
    assert err < 0.85 * err0


def test_non_finite_inputs_are_reported_and_leave_a_consistent_gate():
    from paper_2410_10503_amd import McrError
    n = 32
    img = dev(f32(synth.random_image(n, 2)), torch.float32)
    bad = img.clone()
    bad[5, 7] = float("nan")
    R = Problem(n, 20, 48, 2, "rigid")
    hr = R.handle(torch.float32)
    with pytest.raises(McrError, match="not finite"):
        hr.register_rigid(0, img, bad)
    P = Problem(n, 20, 48, 2, "field")
    for call in (lambda h: h.register_field(0, img, bad), lambda h: h.register_affine(0, img, bad)):
        h = P.handle(torch.float32)
        with pytest.raises(McrError, match="reset to the identity"):
            call(h)
        assert torch.equal(h.warp(0, img), img)
        # the handle stays usable: the other gate's operator pair still runs
        s = h.apply_Ai(1, img)
        assert torch.isfinite(h.apply_Ai_adjoint(1, s)).all()
