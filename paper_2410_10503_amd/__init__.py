"""Motion-compensated SPDHG / PDHG reconstruction on AMD Instinct MI355X.

Python binding of libmcr (include/mcr.h). Every step of the reconstruction
runs in the library's HIP kernels; this module only checks and marshals
arguments (torch tensors on the HIP device provide memory and the stream).

    h = Handle(n, n_angles, n_det, motion=[("rigid", (phi, tx, ty)), ...])
    s = h.apply_Ai(gate, x)             # A D_i x
    b = h.apply_Ai_adjoint(gate, s)     # D_i^T A^T s
    st = h.zero_state()
    h.spdhg_epoch(st, d, alpha, sigma, tau, theta, p, gate_seq)   # Algorithm 1
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib
from ._lib import McrError  # noqa: F401

__all__ = ["Handle", "BatchHandle", "ReconState", "McrError", "step_sizes", "step_sizes_blocks", "project_noalloc"]

_DTYPES = {torch.float32: _lib.MCR_F32, torch.float64: _lib.MCR_F64}


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dbl_array(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * len(vals))(*vals)


def project_noalloc(x, n_angles: int, n_det: int, out):
    """A x into the caller's float32 tensor `out` [n_angles][n_det] with no
    handle and no device allocation (mcr_project_noalloc), on the current
    stream of x's device. x: contiguous float32 [n][n] on the HIP device."""
    n = x.shape[0] if x.dim() == 2 else -1
    for t, shape, name in ((x, (n, n), "x"), (out, (n_angles, n_det), "out")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise ValueError(f"{name} must be a tensor on the HIP device")
        if t.dtype != torch.float32 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape}")
    if out.device != x.device:
        raise ValueError("x and out must be on the same device")
    geo = _lib.Geometry(n, int(n_angles), int(n_det))
    with torch.cuda.device(x.device):
        _lib.check(_lib.load().mcr_project_noalloc(ctypes.byref(geo), x.data_ptr(), out.data_ptr(),
                                                   ctypes.c_void_p(_stream_ptr(x.device))))
    return out


def step_sizes(algo: str, norms_sq: Sequence[float], alpha: float, n_gates: int):
    """Step sizes attaining Theorem 1's rates (host arithmetic in the library).

    algo "spdhg": norms_sq = |A_i|^2 per gate; "pdhg": norms_sq = [|(A_1; ...; A_N)|^2].
    Returns (sigma list, tau, theta, rate per epoch)."""
    lib = _lib.load()
    a = {"spdhg": 0, "pdhg": 1}[algo]
    sig = (ctypes.c_double * n_gates)()
    tau, theta, rate = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.mcr_step_sizes(a, n_gates, _dbl_array(norms_sq), float(alpha), sig,
                                  ctypes.byref(tau), ctypes.byref(theta), ctypes.byref(rate)))
    return list(sig), tau.value, theta.value, rate.value


def step_sizes_blocks(norms_sq: Sequence[float], alpha: float, n_gates: int, n_subsets: int):
    """Step sizes for serial uniform sampling over gates x angle subsets
    (norms_sq: |A_b|^2 per block b = gate * M + subset). Returns
    (sigma list [N M], tau, theta, rate per epoch)."""
    lib = _lib.load()
    nb = n_gates * n_subsets
    if len(norms_sq) != nb:
        raise ValueError(f"need {nb} block norms")
    sig = (ctypes.c_double * nb)()
    tau, theta, rate = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.mcr_step_sizes_blocks(n_gates, n_subsets, _dbl_array(norms_sq), float(alpha), sig,
                                         ctypes.byref(tau), ctypes.byref(theta), ctypes.byref(rate)))
    return list(sig), tau.value, theta.value, rate.value


class ReconState:
    """(x, y_1..y_N, z, z-bar) of Algorithm 1 as device tensors."""

    def __init__(self, x, y, z, zbar):
        self.x, self.y, self.z, self.zbar = x, list(y), z, zbar

    def clone(self):
        return ReconState(self.x.clone(), [v.clone() for v in self.y], self.z.clone(), self.zbar.clone())

    def _c(self):
        ys = (ctypes.c_void_p * len(self.y))(*[v.data_ptr() for v in self.y])
        st = _lib.State(self.x.data_ptr(), self.z.data_ptr(), self.zbar.data_ptr(), ys)
        st._keep = ys
        return st


class Handle:
    """One reconstruction problem: geometry, the gates' motion, workspaces.

    motion: sequence of "identity", ("rigid", (phi_rad, t_x, t_y)) or
    ("field", tensor [2][n][n] float32 on the device).
    """

    def __init__(self, n: int, n_angles: int, n_det: int, motion, dtype=torch.float32, device="cuda"):
        self._lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on the HIP device only")
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be float32 or float64, not {dtype}")
        self.n, self.n_angles, self.n_det = int(n), int(n_angles), int(n_det)
        self.dtype = dtype
        self.n_gates = len(motion)
        self.n_subsets = 1
        self._h = ctypes.c_void_p()
        arr = (_lib.Motion * self.n_gates)()
        keep = []
        for i, m in enumerate(motion):
            arr[i] = self._motion(m, keep)
        self._kinds = [arr[i].kind for i in range(self.n_gates)]
        # bumped by every call that changes a gate's motion; `_installed` is the
        # whole-handle motion last installed by the differentiation path
        # ((kind, tensor) or None when unknown), so that its backward pass can
        # put back what it found
        self._motion_gen = 0
        self._installed = None
        geo = _lib.Geometry(self.n, self.n_angles, self.n_det)
        self._stream = _stream_ptr(self.device)
        _lib.check(self._lib.mcr_create(ctypes.byref(geo), self.n_gates, arr, _DTYPES[dtype],
                                        ctypes.c_void_p(self._stream), ctypes.byref(self._h)))

    def _motion(self, m, keep):
        if m == "identity" or m is None:
            return _lib.Motion(_lib.MOTION_IDENTITY, (ctypes.c_double * 3)(0, 0, 0), None)
        kind, val = m
        if kind == "rigid":
            return _lib.Motion(_lib.MOTION_RIGID, (ctypes.c_double * 3)(*[float(v) for v in val]), None)
        if kind == "field":
            f = val
            if not (isinstance(f, torch.Tensor) and f.dtype == torch.float32 and f.is_cuda
                    and tuple(f.shape) == (2, self.n, self.n)):
                raise ValueError("a field must be a float32 device tensor of shape [2][n][n]")
            f = f.contiguous()
            keep.append(f)
            return _lib.Motion(_lib.MOTION_FIELD, (ctypes.c_double * 3)(0, 0, 0), f.data_ptr())
        raise ValueError(f"unknown motion {kind!r}")

    def close(self):
        if self._h:
            self._lib.mcr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument marshalling ------------------------------------------------
    def _sync_stream(self):
        s = _stream_ptr(self.device)
        if s != self._stream:
            _lib.check(self._lib.mcr_set_stream(self._h, ctypes.c_void_p(s)))
            self._stream = s

    def _check(self, t, shape, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise ValueError(f"{name} must be a tensor on the HIP device")
        if t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {shape}")
        return t.data_ptr()

    def _img(self, t, name="image"):
        return self._check(t, (self.n, self.n), name)

    def _sino(self, t, name="sinogram"):
        return self._check(t, (self.n_angles, self.n_det), name)

    def new_image(self):
        return torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)

    def new_sino(self):
        return torch.empty((self.n_angles, self.n_det), dtype=self.dtype, device=self.device)

    def zero_state(self) -> ReconState:
        z = lambda shape: torch.zeros(shape, dtype=self.dtype, device=self.device)  # noqa: E731
        return ReconState(z((self.n, self.n)), [z((self.n_angles, self.n_det)) for _ in range(self.n_gates)],
                          z((self.n, self.n)), z((self.n, self.n)))

    def _ptrs(self, ts, kind):
        if len(ts) != self.n_gates:
            raise ValueError(f"need {self.n_gates} {kind} arrays, got {len(ts)}")
        vals = [self._sino(t, kind) for t in ts]
        return (ctypes.c_void_p * len(vals))(*vals)

    # -- operators -----------------------------------------------------------
    def _motion_changed(self):
        self._motion_gen += 1
        self._installed = None

    def set_motion(self, gate: int, motion):
        keep = []
        m = self._motion(motion, keep)
        self._motion_changed()
        self._checked_motion_call(gate, lambda: self._lib.mcr_set_motion(self._h, int(gate), ctypes.byref(m)))
        self._kinds[int(gate)] = m.kind

    def _checked_motion_call(self, gate, call):
        """Runs a call that installs a gate's motion; a field rejected by the
        gather-window check, or a registration that fails after its start,
        leaves the gate at the identity."""
        try:
            _lib.check(call())
        except _lib.McrError as e:
            if "reset to the identity" in str(e):
                self._kinds[int(gate)] = _lib.MOTION_IDENTITY
            raise

    def set_rigid_params(self, params):
        """All gates' rigid (phi, t_x, t_y) at once, [N][3]; queued on the stream."""
        vals = [float(v) for row in params for v in row]
        if len(vals) != 3 * self.n_gates:
            raise ValueError(f"need {self.n_gates} x 3 rigid parameters")
        self._sync_stream()
        self._motion_changed()
        _lib.check(self._lib.mcr_set_rigid_params(self._h, _dbl_array(vals)))

    def warp(self, gate, x, out=None):
        self._sync_stream()
        out = self.new_image() if out is None else out
        _lib.check(self._lib.mcr_warp(self._h, int(gate), self._img(x, "x"), self._img(out, "out")))
        return out

    def warp_adjoint(self, gate, b, out=None):
        self._sync_stream()
        out = self.new_image() if out is None else out
        _lib.check(self._lib.mcr_warp_adjoint(self._h, int(gate), self._img(b, "b"), self._img(out, "out")))
        return out

    def project(self, x, out=None):
        self._sync_stream()
        out = self.new_sino() if out is None else out
        _lib.check(self._lib.mcr_project(self._h, self._img(x, "x"), self._sino(out, "out")))
        return out

    def backproject(self, s, out=None):
        self._sync_stream()
        out = self.new_image() if out is None else out
        _lib.check(self._lib.mcr_backproject(self._h, self._sino(s, "s"), self._img(out, "out")))
        return out

    def apply_Ai(self, gate, x, out=None):
        self._sync_stream()
        out = self.new_sino() if out is None else out
        _lib.check(self._lib.mcr_apply_Ai(self._h, int(gate), self._img(x, "x"), self._sino(out, "out")))
        return out

    def apply_Ai_adjoint(self, gate, s, out=None):
        self._sync_stream()
        out = self.new_image() if out is None else out
        _lib.check(self._lib.mcr_apply_Ai_adjoint(self._h, int(gate), self._sino(s, "s"), self._img(out, "out")))
        return out

    # -- Algorithm 1 ---------------------------------------------------------
    def _state(self, st: ReconState):
        self._img(st.x, "x")
        self._img(st.z, "z")
        self._img(st.zbar, "zbar")
        self._ptrs(st.y, "y")
        return st._c()

    def spdhg_iterate(self, st: ReconState, d, alpha, sigma, tau, theta, p, gate_seq):
        self._sync_stream()
        seq = [int(g) for g in gate_seq]
        c_seq = (ctypes.c_int32 * max(1, len(seq)))(*seq)
        _lib.check(self._lib.mcr_spdhg_iterate(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                               float(alpha), _dbl_array(sigma), float(tau), float(theta),
                                               _dbl_array(p), c_seq, len(seq)))

    def spdhg_epoch(self, st: ReconState, d, alpha, sigma, tau, theta, p, gate_seq):
        self._sync_stream()
        seq = [int(g) for g in gate_seq]
        if len(seq) != self.n_gates:
            raise ValueError(f"an epoch has {self.n_gates} iterations, got {len(seq)} gates")
        c_seq = (ctypes.c_int32 * len(seq))(*seq)
        _lib.check(self._lib.mcr_spdhg_epoch(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                             float(alpha), _dbl_array(sigma), float(tau), float(theta),
                                             _dbl_array(p), c_seq))

    def pdhg_epoch(self, st: ReconState, d, alpha, sigma, tau, theta):
        self._sync_stream()
        _lib.check(self._lib.mcr_pdhg_epoch(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                            float(alpha), _dbl_array(sigma), float(tau), float(theta)))

    # -- differentiation ----------------------------------------------------
    def spdhg_iterate_ckpt(self, st: ReconState, d, alpha, sigma, tau, theta, p, gate_seq, x1_ckpt, y_ckpt,
                           b_ckpt=None):
        """spdhg_iterate that also stores, per iteration, x after step (i) and the drawn gate's old dual
        (and, if b_ckpt is given, the iteration's backprojection, which spares the reverse step its
        recomputation)."""
        self._sync_stream()
        seq = [int(g) for g in gate_seq]
        if len(x1_ckpt) != len(seq) or len(y_ckpt) != len(seq) or (b_ckpt is not None and len(b_ckpt) != len(seq)):
            raise ValueError("one checkpoint of each kind per iteration")
        c_seq = (ctypes.c_int32 * max(1, len(seq)))(*seq)
        xs = (ctypes.c_void_p * max(1, len(seq)))(*[self._img(t, "x1_ckpt") for t in x1_ckpt])
        ys = (ctypes.c_void_p * max(1, len(seq)))(*[self._sino(t, "y_ckpt") for t in y_ckpt])
        bs = None if b_ckpt is None else (ctypes.c_void_p * max(1, len(seq)))(*[self._img(t, "b_ckpt")
                                                                                for t in b_ckpt])
        _lib.check(self._lib.mcr_spdhg_iterate_ckpt(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                                    float(alpha), _dbl_array(sigma), float(tau), float(theta),
                                                    _dbl_array(p), c_seq, len(seq), xs, ys, bs))

    def _grad_motion_ptr(self, gate, gm):
        if gm is None:
            return None
        kind = self._kinds[int(gate)]
        if kind == _lib.MOTION_RIGID:
            if not (gm.dtype == torch.float64 and gm.is_cuda and gm.numel() == 3 and gm.is_contiguous()):
                raise ValueError("a rigid motion gradient is a contiguous float64 device tensor of 3 values")
        elif kind == _lib.MOTION_FIELD:
            if not (gm.dtype == self.dtype and gm.is_cuda and tuple(gm.shape) == (2, self.n, self.n)
                    and gm.is_contiguous()):
                raise ValueError(f"a field gradient is a contiguous {self.dtype} device tensor [2][n][n]")
        return gm.data_ptr()

    def spdhg_step_backward(self, gate, x1, y_before, d_gate, alpha, sigma_g, tau, theta, p_g, gx, gy, gz, gzbar,
                            grad_motion=None, b_ckpt=None):
        """Reverse of one SPDHG iteration (adjoints updated in place, motion gradient accumulated);
        b_ckpt: the iteration's stored backprojection, or None to recompute it."""
        self._sync_stream()
        _lib.check(self._lib.mcr_spdhg_step_backward(
            self._h, int(gate), self._img(x1, "x1"), self._sino(y_before, "y_before"), self._sino(d_gate, "d_gate"),
            float(alpha), float(sigma_g), float(tau), float(theta), float(p_g), self._img(gx, "gx"),
            self._sino(gy, "gy"), self._img(gz, "gz"), self._img(gzbar, "gzbar"),
            self._grad_motion_ptr(gate, grad_motion), None if b_ckpt is None else self._img(b_ckpt, "b_ckpt")))

    def warp_motion_grad(self, gate, img, v, grad_motion):
        """grad_motion += d/d(motion of gate) <img, D_gate v>."""
        self._sync_stream()
        _lib.check(self._lib.mcr_warp_motion_grad(self._h, int(gate), self._img(img, "img"), self._img(v, "v"),
                                                  self._grad_motion_ptr(gate, grad_motion)))

    def register_rigid(self, gate: int, ref, target, params=(0.0, 0.0, 0.0), max_iter: int = 200,
                       tol: float = 1e-6):
        """Rigid parameters (phi, t_x, t_y) of `gate` minimising |D ref - target|^2 / 2, from
        `params`; the gate's motion is set to them. Returns (params, energy, steps)."""
        self._sync_stream()
        self._motion_changed()
        th = (ctypes.c_double * 3)(*[float(v) for v in params])
        E, k = ctypes.c_double(), ctypes.c_int32()
        _lib.check(self._lib.mcr_register_rigid(self._h, int(gate), self._img(ref, "ref"), self._img(target, "target"),
                                                th, int(max_iter), float(tol), ctypes.byref(E), ctypes.byref(k)))
        return (th[0], th[1], th[2]), E.value, k.value

    def register_affine(self, gate: int, ref, target, params=(0.0,) * 6, max_iter: int = 300,
                        tol: float = 1e-6):
        """Affine displacement field u = A (p - c) + t of field gate `gate`, params (A00, A01, A10,
        A11, t_x, t_y), minimising |D ref - target|^2 / 2 from `params`; the gate's field is set to
        it. Returns (params, energy, steps)."""
        self._sync_stream()
        self._motion_changed()
        th = (ctypes.c_double * 6)(*[float(v) for v in params])
        E, k = ctypes.c_double(), ctypes.c_int32()
        rp, tp = self._img(ref, "ref"), self._img(target, "target")
        self._checked_motion_call(gate, lambda: self._lib.mcr_register_affine(
            self._h, int(gate), rp, tp, th, int(max_iter), float(tol), ctypes.byref(E), ctypes.byref(k)))
        return tuple(th[m] for m in range(6)), E.value, k.value

    def register_field(self, gate: int, ref, target, field=None, lam: float = 0.01, max_iter: int = 300,
                       tol: float = 1e-4, sigmas=()):
        """Dense displacement field of field gate `gate` minimising |D_u ref - target|^2 / 2 +
        lam / 2 R(u) (R: squared differences of adjacent pixels), from `field` (float32 [2][n][n]
        device tensor, overwritten with the result; zero if None); the gate's field is set to it.
        sigmas: scale-space schedule (Gaussian widths in pixels, coarse to fine; empty: one level
        on the images themselves). Returns (field, energy, steps)."""
        self._sync_stream()
        self._motion_changed()
        if field is None:
            field = torch.zeros((2, self.n, self.n), dtype=torch.float32, device=self.device)
        if not (isinstance(field, torch.Tensor) and field.dtype == torch.float32 and field.is_cuda
                and tuple(field.shape) == (2, self.n, self.n) and field.is_contiguous()):
            raise ValueError("field must be a contiguous float32 device tensor of shape [2][n][n]")
        E, k = ctypes.c_double(), ctypes.c_int32()
        rp, tp = self._img(ref, "ref"), self._img(target, "target")
        sg = [float(v) for v in sigmas]
        sga = (ctypes.c_double * max(1, len(sg)))(*sg)
        self._checked_motion_call(gate, lambda: self._lib.mcr_register_field(
            self._h, int(gate), rp, tp, field.data_ptr(), float(lam), sga, len(sg), int(max_iter), float(tol),
            ctypes.byref(E), ctypes.byref(k)))
        return field, E.value, k.value

    # -- FP64 diagnostics ----------------------------------------------------
    def power_norm_sq(self, gate: int, v0, max_iter: int = 500, rtol: float = 1e-12):
        """|A_gate|^2 (gate >= 0) or the stacked |(A_1; ...; A_N)|^2 (gate = -1)."""
        self._sync_stream()
        if not (v0.dtype == torch.float64 and v0.is_cuda and tuple(v0.shape) == (self.n, self.n)
                and v0.is_contiguous()):
            raise ValueError("v0 must be a contiguous float64 device tensor of shape (n, n)")
        out, it = ctypes.c_double(), ctypes.c_int32()
        _lib.check(self._lib.mcr_power_norm_sq(self._h, int(gate), v0.data_ptr(), int(max_iter), float(rtol),
                                               ctypes.byref(out), ctypes.byref(it)))
        return out.value, it.value

    def set_subsets(self, n_subsets: int, paired: bool = False):
        """Cut the angles into n_subsets subsets (gates x angle-subsets
        sampling): contiguous ranges, or (paired) ranges of the first half
        with their partners a quarter turn away."""
        self._sync_stream()
        _lib.check(self._lib.mcr_set_subset_partition(self._h, int(n_subsets), 1 if paired else 0))
        self.n_subsets = int(n_subsets)

    def block_norm_sq(self, gate: int, subset: int, v0, max_iter: int = 500, rtol: float = 1e-12):
        """|A_b|^2 of block (gate, subset)."""
        self._sync_stream()
        if not (v0.dtype == torch.float64 and v0.is_cuda and tuple(v0.shape) == (self.n, self.n)
                and v0.is_contiguous()):
            raise ValueError("v0 must be a contiguous float64 device tensor of shape (n, n)")
        out, it = ctypes.c_double(), ctypes.c_int32()
        _lib.check(self._lib.mcr_block_norm_sq(self._h, int(gate), int(subset), v0.data_ptr(), int(max_iter),
                                               float(rtol), ctypes.byref(out), ctypes.byref(it)))
        return out.value, it.value

    def spdhg_blocks_iterate(self, st: ReconState, d, alpha, sigma, tau, theta, p, block_seq):
        """Iterations of Algorithm 1 over blocks b = gate * M + subset (sigma, p per block)."""
        self._sync_stream()
        nb = self.n_gates * self.n_subsets
        if len(sigma) != nb or len(p) != nb:
            raise ValueError(f"sigma and p need {nb} entries (one per block)")
        seq = [int(b) for b in block_seq]
        c_seq = (ctypes.c_int32 * max(1, len(seq)))(*seq)
        _lib.check(self._lib.mcr_spdhg_blocks_iterate(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                                      float(alpha), _dbl_array(sigma), float(tau), float(theta),
                                                      _dbl_array(p), c_seq, len(seq)))

    def objective(self, x, d, alpha) -> float:
        self._sync_stream()
        out = ctypes.c_double()
        _lib.check(self._lib.mcr_objective(self._h, self._img(x, "x"), self._ptrs(d, "d"), float(alpha),
                                           ctypes.byref(out)))
        return out.value

    def duality_gap(self, st: ReconState, d, alpha) -> float:
        self._sync_stream()
        out = ctypes.c_double()
        _lib.check(self._lib.mcr_duality_gap(self._h, ctypes.byref(self._state(st)), self._ptrs(d, "d"),
                                             float(alpha), ctypes.byref(out)))
        return out.value

    def autotune(self, gates_per_launch: int = 1):
        """Pick the fastest float32 projector-pair variants for this geometry;
        returns {"fwd": ..., "adj_px": ..., "adj_shares": ...}."""
        self._sync_stream()
        f, p, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.mcr_autotune(self._h, int(gates_per_launch), ctypes.byref(f), ctypes.byref(p),
                                          ctypes.byref(s)))
        return {"fwd": f.value, "adj_px": p.value, "adj_shares": s.value}

    def set_variant(self, fwd: int, adj_px: int, adj_shares: int):
        _lib.check(self._lib.mcr_set_variant(self._h, int(fwd), int(adj_px), int(adj_shares)))

    def profile(self, enable: bool = True):
        """Bracket every kernel launch with HIP events (see profile_read)."""
        _lib.check(self._lib.mcr_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read; synchronises."""
        k = len(_lib.KERNEL_CLASSES)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        _lib.check(self._lib.mcr_profile_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.KERNEL_CLASSES)}

    def info(self):
        geo, ng, dt, rad = _lib.Geometry(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.mcr_get_info(self._h, ctypes.byref(geo), ctypes.byref(ng), ctypes.byref(dt),
                                          ctypes.byref(rad)))
        return {"n": geo.n, "n_angles": geo.n_angles, "n_det": geo.n_det, "n_gates": ng.value,
                "dtype": dt.value, "window_radius": rad.value}


class BatchHandle(Handle):
    """S independent slices sharing one geometry, advanced one SPDHG epoch per
    call (all slices together; optionally replayed as a HIP graph).

    gates_per_slice: list of N_s; motion: one entry per gate, slice after
    slice. State: x, z, zbar [S][n][n]; y [sum N_s][n_angles][n_det]."""

    def __init__(self, n: int, n_angles: int, n_det: int, gates_per_slice, motion, dtype=torch.float32,
                 device="cuda"):
        self._lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on the HIP device only")
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be float32 or float64, not {dtype}")
        self.n, self.n_angles, self.n_det = int(n), int(n_angles), int(n_det)
        self.dtype = dtype
        self.gates_per_slice = [int(v) for v in gates_per_slice]
        self.n_slices = len(self.gates_per_slice)
        self.n_gates = sum(self.gates_per_slice)
        self.offsets = [sum(self.gates_per_slice[:s]) for s in range(self.n_slices)]
        if len(motion) != self.n_gates:
            raise ValueError(f"need {self.n_gates} motion entries, got {len(motion)}")
        self._h = ctypes.c_void_p()
        arr = (_lib.Motion * self.n_gates)()
        keep = []
        for i, m in enumerate(motion):
            arr[i] = self._motion(m, keep)
        self._kinds = [arr[i].kind for i in range(self.n_gates)]
        # bumped by every call that changes a gate's motion; `_installed` is the
        # whole-handle motion last installed by the differentiation path
        # ((kind, tensor) or None when unknown), so that its backward pass can
        # put back what it found
        self._motion_gen = 0
        self._installed = None
        geo = _lib.Geometry(self.n, self.n_angles, self.n_det)
        ng = (ctypes.c_int32 * self.n_slices)(*self.gates_per_slice)
        self._stream = _stream_ptr(self.device)
        _lib.check(self._lib.mcr_batch_create(ctypes.byref(geo), self.n_slices, ng, arr, _DTYPES[dtype],
                                              ctypes.c_void_p(self._stream), ctypes.byref(self._h)))

    def zero_batch_state(self):
        z = lambda *shape: torch.zeros(shape, dtype=self.dtype, device=self.device)  # noqa: E731
        S, n = self.n_slices, self.n
        return {"x": z(S, n, n), "z": z(S, n, n), "zbar": z(S, n, n),
                "y": z(self.n_gates, self.n_angles, self.n_det)}

    def _batch_arr(self, t, shape, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == self.dtype and tuple(t.shape) == shape
                and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} device tensor of shape {shape}")
        return t.data_ptr()

    def batch_spdhg_epoch(self, st, d, alpha, sigma, tau, theta, p, gate_seq, use_graph: bool = True):
        """alpha, tau, theta: per slice; sigma, p, gate_seq: per gate (global order);
        gate_seq holds each slice's N_s local draws at the slice's first gate."""
        self._sync_stream()
        S, n, G = self.n_slices, self.n, self.n_gates
        img = (S, n, n)
        sino = (G, self.n_angles, self.n_det)
        seq = [int(v) for v in gate_seq]
        if len(seq) != G or len(sigma) != G or len(p) != G or len(alpha) != S or len(tau) != S or len(theta) != S:
            raise ValueError("per-slice arrays need S entries and per-gate arrays sum(N_s)")
        _lib.check(self._lib.mcr_batch_spdhg_epoch(
            self._h, self._batch_arr(st["x"], img, "x"), self._batch_arr(st["z"], img, "z"),
            self._batch_arr(st["zbar"], img, "zbar"), self._batch_arr(st["y"], sino, "y"),
            self._batch_arr(d, sino, "d"), _dbl_array(alpha), _dbl_array(sigma), _dbl_array(tau),
            _dbl_array(theta), _dbl_array(p), (ctypes.c_int32 * G)(*seq), 1 if use_graph else 0))
