"""torch.autograd through unrolled SPDHG iterations (Algorithm 1).

`unrolled_spdhg(handle, x0, motion, d, alpha, sigma, tau, theta, p, gate_seq)`
runs len(gate_seq) SPDHG iterations from (x0, y = 0, z = 0, z-bar = 0) with
the given motion and returns the final image. Gradients flow to x0 and to the
motion parameters: a [N][3] float64 tensor of rigid (phi, t_x, t_y) or a
[N][2][n][n] tensor of displacement fields. The forward pass keeps one
checkpoint per iteration (the image after step (i), the drawn gate's old
dual and the iteration's backprojection); the backward pass runs the
library's reverse of each iteration (mcr_spdhg_step_backward) from its
checkpoint. All arithmetic runs in the
library's kernels; this module moves tensors.

The handle holds one motion at a time. The forward pass installs its motion
and keeps a copy; if the handle's motion has changed by the time backward runs
(another unrolled forward on the same handle, a finite-difference evaluation,
a registration), backward installs the copy for its reverse steps, so the
gradient is that of its own operators A_i = A D_i, and then puts back the
motion it found when that motion was installed by another unrolled forward
(otherwise the forward's motion stays installed).
"""
from __future__ import annotations

import torch


def _apply_motion(handle, kind: str, motion: torch.Tensor):
    """Installs the whole-handle motion and records it (with the handle's
    motion generation after the change)."""
    if kind == "rigid":
        handle.set_rigid_params(motion.detach().to(torch.float64).cpu().tolist())
    else:
        for i in range(handle.n_gates):
            handle.set_motion(i, ("field", motion[i].detach().to(torch.float32).contiguous()))
    handle._installed = (kind, motion)
    return handle._motion_gen


class UnrolledSPDHG(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, motion, handle, kind, d, alpha, sigma, tau, theta, p, gate_seq):
        saved = motion.detach().clone()
        ctx.motion_gen = _apply_motion(handle, kind, saved)
        ctx.motion_saved = saved
        st = handle.zero_state()
        st.x.copy_(x0.detach())
        K = len(gate_seq)
        x1c = [handle.new_image() for _ in range(K)]
        yc = [handle.new_sino() for _ in range(K)]
        bc = [handle.new_image() for _ in range(K)]  # spares the reverse steps a recomputation each
        handle.spdhg_iterate_ckpt(st, d, alpha, sigma, tau, theta, p, gate_seq, x1c, yc, bc)
        ctx.handle, ctx.kind = handle, kind
        ctx.args = (list(d), alpha, list(sigma), tau, theta, list(p), [int(g) for g in gate_seq])
        ctx.ckpt = (x1c, yc, bc)
        ctx.motion_shape = tuple(motion.shape)
        ctx.motion_device = motion.device
        ctx.motion_dtype = motion.dtype
        return st.x

    @staticmethod
    def backward(ctx, gout):
        h = ctx.handle
        d, alpha, sigma, tau, theta, p, seq = ctx.args
        x1c, yc, bc = ctx.ckpt
        restore = None
        if h._motion_gen != ctx.motion_gen:
            restore = h._installed
            _apply_motion(h, ctx.kind, ctx.motion_saved)
        gx = gout.detach().to(h.dtype).contiguous().clone()
        gz = torch.zeros_like(gx)
        gzb = torch.zeros_like(gx)
        gy = {}
        if ctx.kind == "rigid":
            gm = torch.zeros((h.n_gates, 3), dtype=torch.float64, device=h.device)
        else:
            gm = torch.zeros((h.n_gates, 2, h.n, h.n), dtype=h.dtype, device=h.device)
        for k in range(len(seq) - 1, -1, -1):
            g = seq[k]
            if g not in gy:
                gy[g] = torch.zeros((h.n_angles, h.n_det), dtype=h.dtype, device=h.device)
            h.spdhg_step_backward(g, x1c[k], yc[k], d[g], alpha, sigma[g], tau, theta, p[g], gx, gy[g], gz, gzb,
                                  gm[g], b_ckpt=bc[k])
        if restore is not None:
            _apply_motion(h, *restore)
        gmot = gm.to(device=ctx.motion_device, dtype=ctx.motion_dtype).reshape(ctx.motion_shape)
        return gx, gmot, None, None, None, None, None, None, None, None, None


def unrolled_spdhg(handle, x0, motion, d, alpha, sigma, tau, theta, p, gate_seq, kind: str | None = None):
    """Final image of len(gate_seq) SPDHG iterations, differentiable in x0 and motion."""
    if kind is None:
        kind = "rigid" if motion.dim() == 2 else "field"
    if kind not in ("rigid", "field"):
        raise ValueError("motion must be rigid [N][3] or fields [N][2][n][n]")
    return UnrolledSPDHG.apply(x0, motion, handle, kind, d, alpha, sigma, tau, theta, p, gate_seq)


__all__ = ["UnrolledSPDHG", "unrolled_spdhg"]
