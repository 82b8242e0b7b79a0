"""Ray transform A: R^{n x n} -> R^{n_angles x n_det}, 2D parallel beam (FP64).

The paper names the ray transform of a 2D parallel geometry (Section II-A, the
forward operator A; Section III, "Description") without fixing a
discretisation. This oracle uses the Joseph rule:

* pixel (r, c) has its centre at x_c = c - (n-1)/2 (columns) and
  y_r = r - (n-1)/2 (rows), unit pixels;
* angle k is theta_k = k*pi/n_angles; detector bin j has its centre at
  t_j = j - (n_det-1)/2, unit spacing; ray (k, j) is the line
  {p : p . (cos theta_k, sin theta_k) = t_j};
* the ray steps along rows when 4k <= n_angles or 4k >= 3 n_angles (that is
  |cos| >= |sin|, with the 45 and 135 degree ties decided by the integer rule),
  otherwise along columns;
* row stepping: in row r the ray crosses column position
  c_f = (t_j - y_r sin) / cos + (n-1)/2 and samples the row by linear
  interpolation between columns floor(c_f) and floor(c_f)+1, pixels outside
  the image being zero; the ray sum is the sum over rows times 1/|cos|;
* column stepping: the same with rows and columns exchanged,
  r_f = (t_j - x_c cos) / sin + (n-1)/2 and weight 1/|sin|.

A^T is the scatter of exactly the same weights (np.bincount), so it is the
exact transpose of `forward` by construction. `sparse_matrix` assembles the
same weights, angle by angle, as a sparse matrix: the matrix of `forward`,
whose transpose is `adjoint` (used where the full-size iterations would
otherwise take hours).
"""
from __future__ import annotations

import numpy as np


def angle_table(n_angles: int):
    """theta_k = k pi / n_angles and the stepping axis (True = rows)."""
    k = np.arange(n_angles)
    theta = np.pi * k / n_angles
    rows = (4 * k <= n_angles) | (4 * k >= 3 * n_angles)
    return theta, rows


def _crossings(n: int, n_det: int, k: int, n_angles: int):
    """For angle k: positions c_f[lane, j] along the interpolation axis, the step
    weight, and whether lanes are image rows (row stepping) or columns."""
    theta = np.pi * k / n_angles
    cs, sn = np.cos(theta), np.sin(theta)
    half = (n - 1) / 2.0
    t = np.arange(n_det) - (n_det - 1) / 2.0
    pos = np.arange(n) - half
    rows = (4 * k <= n_angles) or (4 * k >= 3 * n_angles)
    if rows:
        cf = (t[None, :] - pos[:, None] * sn) / cs + half
        ds = 1.0 / abs(cs)
    else:
        cf = (t[None, :] - pos[:, None] * cs) / sn + half
        ds = 1.0 / abs(sn)
    return cf, ds, rows


def forward(x: np.ndarray, n_angles: int, n_det: int) -> np.ndarray:
    """A x for a square image x [n][n]; returns [n_angles][n_det] float64."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    assert x.shape == (n, n)
    padded = np.zeros((n + 2, n + 2))
    padded[1:n + 1, 1:n + 1] = x
    lane = np.arange(n)[:, None]
    out = np.empty((n_angles, n_det))
    for k in range(n_angles):
        cf, ds, rows = _crossings(n, n_det, k, n_angles)
        img = padded if rows else padded.T     # img[lane+1, pos+1]
        c0 = np.floor(cf)
        f = cf - c0
        inside = (c0 >= -1) & (c0 <= n - 1)
        ci = np.clip(c0, -1, n - 1).astype(np.int64)
        samp = (1.0 - f) * img[lane + 1, ci + 1] + f * img[lane + 1, ci + 2]
        out[k] = ds * np.where(inside, samp, 0.0).sum(axis=0)
    return out


def adjoint(y: np.ndarray, n: int) -> np.ndarray:
    """A^T y for a sinogram y [n_angles][n_det]; returns [n][n] float64."""
    y = np.asarray(y, dtype=np.float64)
    n_angles, n_det = y.shape
    lane = np.broadcast_to(np.arange(n)[:, None], (n, n_det))
    acc = np.zeros(n * n)
    for k in range(n_angles):
        cf, ds, rows = _crossings(n, n_det, k, n_angles)
        c0 = np.floor(cf).astype(np.int64)
        f = cf - c0
        yk = ds * np.broadcast_to(y[k][None, :], cf.shape)
        for tap, w in ((c0, (1.0 - f) * yk), (c0 + 1, f * yk)):
            ok = (tap >= 0) & (tap < n)
            idx = (lane * n + tap) if rows else (tap * n + lane)
            acc += np.bincount(idx[ok], weights=w[ok], minlength=n * n)
    return acc.reshape(n, n)


def ray_sum(x: np.ndarray, n_angles: int, n_det: int, k: int, j: int) -> float:
    """(A x)[k, j] for one ray, by the same rule as `forward` (for sampled checks
    at sizes where the full transform is slow)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    cf, ds, rows = _crossings(n, n_det, k, n_angles)
    cf = cf[:, j]
    img = x if rows else x.T
    c0 = np.floor(cf).astype(np.int64)
    f = cf - c0
    total = 0.0
    for lane in range(n):
        for tap, w in ((c0[lane], 1.0 - f[lane]), (c0[lane] + 1, f[lane])):
            if 0 <= tap < n:
                total += w * img[lane, tap]
    return ds * total


def backproject_pixel(y: np.ndarray, n: int, r: int, c: int) -> float:
    """(A^T y)[r, c] for one pixel: the sum over all rays of the ray's weight on
    this pixel (the hat function of the crossing distance) times y."""
    y = np.asarray(y, dtype=np.float64)
    n_angles, n_det = y.shape
    total = 0.0
    for k in range(n_angles):
        cf, ds, rows = _crossings(n, n_det, k, n_angles)
        lane, target = (r, c) if rows else (c, r)
        w = np.maximum(0.0, 1.0 - np.abs(cf[lane] - target))
        total += ds * float(np.dot(w, y[k]))
    return total


def matrix(n: int, n_angles: int, n_det: int) -> np.ndarray:
    """Dense matrix of `forward` by columns (tiny sizes only)."""
    m = np.zeros((n_angles * n_det, n * n))
    e = np.zeros(n * n)
    for q in range(n * n):
        e[:] = 0.0
        e[q] = 1.0
        m[:, q] = forward(e.reshape(n, n), n_angles, n_det).ravel()
    return m


def sparse_matrix(n: int, n_angles: int, n_det: int):
    """The matrix of `forward` (rows: rays k * n_det + j; columns: pixels
    r * n + c) as a scipy.sparse CSR matrix, assembled from the same crossings
    and weights: ray (k, j) holds, for every line along its stepping axis,
    weight ds (1 - f) on the pixel at floor(c_f) and ds f on the next one,
    where those pixels lie inside the image. A ray meets each pixel of a line
    at most once, so no entry is written twice."""
    import scipy.sparse as sps
    lane = np.arange(n)[:, None]
    counts = np.zeros(n_angles * n_det, dtype=np.int64)
    cols, vals = [], []
    for k in range(n_angles):
        cf, ds, rows = _crossings(n, n_det, k, n_angles)
        c0 = np.floor(cf).astype(np.int64)
        f = cf - c0
        # entries of this angle ordered by ray, then line, then tap
        tap = np.stack([c0, c0 + 1], axis=-1)                       # [lane][ray][2]
        w = np.stack([ds * (1.0 - f), ds * f], axis=-1)
        pix = (lane[..., None] * n + tap) if rows else (tap * n + lane[..., None])
        ok = (tap >= 0) & (tap < n)
        order = (1, 0, 2)                                          # -> [ray][lane][2]
        ok_t = ok.transpose(order)
        cols.append(pix.transpose(order)[ok_t].astype(np.int32))
        vals.append(w.transpose(order)[ok_t])
        counts[k * n_det:(k + 1) * n_det] = ok_t.reshape(n_det, -1).sum(axis=1)
    indptr = np.zeros(n_angles * n_det + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    indices = np.concatenate(cols)
    del cols
    data = np.concatenate(vals)
    del vals
    if indptr[-1] < 2 ** 31:
        indptr = indptr.astype(np.int32)
    return sps.csr_matrix((data, indices, indptr), shape=(n_angles * n_det, n * n))
