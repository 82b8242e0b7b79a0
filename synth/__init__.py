"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws numbers and rasterises shapes; it holds none of the
reconstruction method's arithmetic (no projector, warp, prox or iteration).
Everything that both the HIP path and the CPU oracle consume comes from here,
rounded to float32 where the paper's data would be measured data:

* phantoms: random-ellipse images and a chest-like image (body ellipse, two
  lungs at 0.2, small nodules), rasterised by the pixel-centre test;
* motion: rigid (rotation about the image centre, translation) and a non-rigid
  displacement field (linear vertical dilatation by gate phase plus smooth
  Gaussian bumps), the two kinds of motion of the paper's experiments
  (Section III, "Description");
* unit-variance Gaussian noise arrays (the caller scales them to the model's
  per-entry variance, Section II-A);
* the serial uniform gate sequence of SPDHG (Algorithm 1, step (ii)), one draw
  per iteration, a pure function of (seed, epoch).

The paper's walnut and chest CT datasets are not available; these generators
stand in for them with the shapes and value ranges of the workloads.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "ellipse_phantom", "chest_phantom", "disc_image",
    "rigid_params", "dilatation_fields", "unit_noise", "gate_sequence",
    "random_image", "random_sinograms", "BatchSlice", "batched_slices",
]


def _rng(*seed):
    return np.random.Generator(np.random.PCG64(list(seed)))


def _grid(n):
    """Pixel-centre coordinates (x = column offset, y = row offset) from the image centre."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return x - c, y - c


def _ellipse_mask(x, y, cx, cy, a, b, phi):
    cp, sp = np.cos(phi), np.sin(phi)
    u = (x - cx) * cp + (y - cy) * sp
    v = -(x - cx) * sp + (y - cy) * cp
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def ellipse_phantom(n: int, seed: int, n_ellipses: int = 10) -> np.ndarray:
    """Sum of `n_ellipses` random ellipses, float32 [n][n].

    Centres uniform in the disc of radius 0.8*n/2, semi-axes U[0.05, 0.4]*n/2,
    orientation U[0, pi), intensity U[0, 1].
    """
    g = _rng(seed, 0xE11)
    x, y = _grid(n)
    img = np.zeros((n, n))
    h = n / 2.0
    for _ in range(n_ellipses):
        r = 0.8 * h * np.sqrt(g.uniform())
        ang = g.uniform(0, 2 * np.pi)
        cx, cy = r * np.cos(ang), r * np.sin(ang)
        a, b = g.uniform(0.05, 0.4, size=2) * h
        phi = g.uniform(0, np.pi)
        val = g.uniform(0, 1)
        img += val * _ellipse_mask(x, y, cx, cy, a, b, phi)
    return img.astype(np.float32)


def chest_phantom(n: int, seed: int) -> np.ndarray:
    """Chest-like slice, float32 [n][n]: body ellipse at 1, two lung ellipses at
    0.2, and 3 to 6 nodules (discs of radius U[3, 8] px at 512, scaled with n) at 1
    inside the lungs."""
    g = _rng(seed, 0xC4E5)
    x, y = _grid(n)
    h = n / 2.0
    img = np.zeros((n, n))
    img[_ellipse_mask(x, y, 0.0, 0.0, 0.85 * h, 0.62 * h, 0.0)] = 1.0
    lungs = [(-0.38 * h, -0.02 * h, 0.27 * h, 0.45 * h, 0.08),
             (0.38 * h, -0.02 * h, 0.27 * h, 0.45 * h, -0.08)]
    for (cx, cy, a, b, phi) in lungs:
        img[_ellipse_mask(x, y, cx, cy, a, b, phi)] = 0.2
    scale = n / 512.0
    for _ in range(int(g.integers(3, 7))):
        cx, cy, a, b, phi = lungs[int(g.integers(0, 2))]
        # a point inside the lung ellipse, away from its rim
        rr = 0.6 * np.sqrt(g.uniform())
        ang = g.uniform(0, 2 * np.pi)
        u, v = rr * a * np.cos(ang), rr * b * np.sin(ang)
        px = cx + u * np.cos(phi) - v * np.sin(phi)
        py = cy + u * np.sin(phi) + v * np.cos(phi)
        rad = max(g.uniform(3.0, 8.0) * scale, 1.0)
        img[(x - px) ** 2 + (y - py) ** 2 <= rad ** 2] = 1.0
    return img.astype(np.float32)


def disc_image(n: int, cx: float, cy: float, radius: float, supersample: int = 4) -> np.ndarray:
    """Uniform disc of value 1, centre (cx, cy) in centred pixel units, area-sampled
    on a supersample x supersample grid per pixel. float64 [n][n]."""
    s = supersample
    x, y = _grid(n)
    acc = np.zeros((n, n))
    off = (np.arange(s) + 0.5) / s - 0.5
    for dy in off:
        for dx in off:
            acc += ((x + dx - cx) ** 2 + (y + dy - cy) ** 2) <= radius ** 2
    return acc / (s * s)


def rigid_params(n_gates: int, seed: int, max_rot_deg: float, max_shift: float) -> np.ndarray:
    """[n_gates][3] = (phi [rad], t_x [px], t_y [px]), each uniform in its range,
    rounded to float32 values (returned as float64)."""
    g = _rng(seed, 0x516)
    phi = np.deg2rad(g.uniform(-max_rot_deg, max_rot_deg, size=n_gates))
    t = g.uniform(-max_shift, max_shift, size=(n_gates, 2))
    out = np.concatenate([phi[:, None], t], axis=1)
    return out.astype(np.float32).astype(np.float64)


def dilatation_fields(n: int, n_gates: int, seed: int, compress_px: float = 8.0,
                      n_bumps: int = 6, bump_sigma: float = 40.0,
                      bump_amp_max: float = 4.0) -> np.ndarray:
    """Non-rigid displacement fields, float32 [n_gates][2][n][n] (plane 0 = u_x
    along columns, plane 1 = u_y along rows, in pixels).

    Gate phase q_i = i/(N-1) (gate 0 is the identity). Vertical linear
    dilatation u_y = compress_px * q_i * y / (n/2) about the centre row, plus
    `n_bumps` Gaussian bumps (std `bump_sigma` px at 512, scaled with n) with
    amplitude U[0, bump_amp_max] px along a random unit direction, centred
    uniformly in the body ellipse, each scaled by q_i.
    """
    g = _rng(seed, 0xF1E1D)
    x, y = _grid(n)
    h = n / 2.0
    scale = n / 512.0
    sig = bump_sigma * scale
    bumps = []
    for _ in range(n_bumps):
        rr = np.sqrt(g.uniform())
        ang = g.uniform(0, 2 * np.pi)
        bx, by = 0.85 * h * rr * np.cos(ang), 0.62 * h * rr * np.sin(ang)
        amp = g.uniform(0, bump_amp_max) * scale
        d = g.uniform(0, 2 * np.pi)
        bumps.append((bx, by, amp * np.cos(d), amp * np.sin(d)))
    base_x = np.zeros((n, n))
    base_y = compress_px * scale * y / h
    for (bx, by, ax, ay) in bumps:
        gsn = np.exp(-((x - bx) ** 2 + (y - by) ** 2) / (2 * sig ** 2))
        base_x = base_x + ax * gsn
        base_y = base_y + ay * gsn
    out = np.zeros((n_gates, 2, n, n))
    for i in range(n_gates):
        q = i / (n_gates - 1) if n_gates > 1 else 0.0
        out[i, 0] = q * base_x
        out[i, 1] = q * base_y
    return out.astype(np.float32)


def unit_noise(shape, seed: int) -> np.ndarray:
    """Standard normal float64 array (scaled by the caller to the model's variance)."""
    return _rng(seed, 0x4015E).standard_normal(shape)


def gate_sequence(n_gates: int, seed: int, epoch: int, length: int | None = None) -> np.ndarray:
    """Serial uniform sampling: `length` (default n_gates) i.i.d. draws from
    {0..n_gates-1}, a pure function of (seed, epoch). int32."""
    m = n_gates if length is None else length
    return _rng(seed, epoch, 0x6A7E).integers(0, n_gates, size=m).astype(np.int32)


def random_image(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    return _rng(seed, 0x1A6).standard_normal((n, n)).astype(dtype)


def random_sinograms(count: int, n_angles: int, n_det: int, seed: int, dtype=np.float32) -> np.ndarray:
    return _rng(seed, 0x5160).standard_normal((count, n_angles, n_det)).astype(dtype)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic problem: image size, parallel-beam sampling, gates, motion, alpha."""
    name: str
    n: int
    n_angles: int
    n_det: int
    n_gates: int
    motion: str            # "rigid" | "field" | "identity"
    alpha: float
    max_rot_deg: float = 0.0
    max_shift: float = 0.0
    phantom: str = "ellipses"   # "ellipses" | "chest"
    phantom_seed: int = 0
    motion_seed: int = 1
    noise_seed: int = 2
    gate_seed: int = 3
    kappa: float = 0.0     # > 0: alpha = |A|^2 / kappa (the paper's regime), computed by the caller

    def image(self) -> np.ndarray:
        if self.phantom == "chest":
            return chest_phantom(self.n, self.phantom_seed)
        return ellipse_phantom(self.n, self.phantom_seed)

    def rigid(self) -> np.ndarray:
        return rigid_params(self.n_gates, self.motion_seed, self.max_rot_deg, self.max_shift)

    def fields(self) -> np.ndarray:
        return dilatation_fields(self.n, self.n_gates, self.motion_seed)


WORKLOADS = {
    # 128^2 FP64 plain SPDHG, 4 rigid gates
    "ellipses128_rigid4": Workload("ellipses128_rigid4", 128, 120, 182, 4, "rigid", 1e-2, 5.0, 4.0),
    # 512^2, 720 x 730, 8 rigid gates (PDHG vs SPDHG)
    "ellipses512_rigid8": Workload("ellipses512_rigid8", 512, 720, 730, 8, "rigid", 1e-3, 8.0, 10.0),
    # 512^2 chest, 720 x 730, 16 non-rigid gates (headline)
    "chest512_field16": Workload("chest512_field16", 512, 720, 730, 16, "field", 1e-3, phantom="chest"),
    # 512^2, 16 rigid gates (differentiable case, and the rigid twin of the headline)
    "ellipses512_rigid16": Workload("ellipses512_rigid16", 512, 720, 730, 16, "rigid", 1e-3, 8.0, 10.0),
    # one slice shape of the batched case
    "ellipses256_slice": Workload("ellipses256_slice", 256, 360, 366, 8, "rigid", 1e-3, 8.0, 10.0),
    # the paper's regime (Section III: kappa = |A|^2 / alpha ~ 70): 20 rigid gates
    # (stand-in for the walnut) and 10 dilatation gates (stand-in for the chest)
    "ellipses128_rigid20_k70": Workload("ellipses128_rigid20_k70", 128, 120, 182, 20, "rigid", 0.0, 5.0, 4.0,
                                        kappa=70.0),
    "chest128_field10_k70": Workload("chest128_field10_k70", 128, 120, 182, 10, "field", 0.0, phantom="chest",
                                     kappa=70.0),
}


@dataclasses.dataclass(frozen=True)
class BatchSlice:
    """One slice of the batched workload: its gate count, kind of motion and
    the seeds of its phantom, motion, noise and gate draws."""
    index: int
    n_gates: int
    motion: str            # "rigid" | "field"
    phantom_seed: int
    motion_seed: int
    noise_seed: int
    gate_seed: int

    def image(self, n: int) -> np.ndarray:
        return ellipse_phantom(n, self.phantom_seed)

    def rigid(self) -> np.ndarray:
        return rigid_params(self.n_gates, self.motion_seed, 8.0, 10.0)

    def fields(self, n: int) -> np.ndarray:
        return dilatation_fields(n, self.n_gates, self.motion_seed)


def batched_slices(count: int = 64, seed: int = 4):
    """The batched workload: `count` independent ellipse slices whose gate
    counts are uniform in {4..32}; odd slices move non-rigidly (dilatation
    fields), even ones rigidly (rotation up to 8 deg, shift up to 10 px)."""
    ngs = np.random.default_rng(seed).integers(4, 33, size=count)
    return [BatchSlice(s, int(ngs[s]), "field" if s % 2 else "rigid", 200 + s, 100 + s, 300 + s, 500 + s)
            for s in range(count)]
