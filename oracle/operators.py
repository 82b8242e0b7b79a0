"""Gated operators A_i = A D_i and A_i^* = D_i^* A^* (Section II-A; Algorithm 1)."""
from __future__ import annotations

import numpy as np

from . import projector, warp


class GatedOperators:
    """The N gate operators of one problem.

    motion: "identity", ("rigid", params [N][3]) or ("field", fields [N][2][n][n]).
    matrix (optional): projector.sparse_matrix(n, n_angles, n_det); A and A^T
    are then its products (the same weights, summed in another order).
    """

    def __init__(self, n: int, n_angles: int, n_det: int, kind: str, params=None, n_gates: int | None = None,
                 matrix=None):
        self.n, self.n_angles, self.n_det = n, n_angles, n_det
        self.kind = kind
        if matrix is not None and matrix.shape != (n_angles * n_det, n * n):
            raise ValueError("matrix shape does not match the geometry")
        self.matrix = matrix
        if kind == "identity":
            self.n_gates = int(n_gates)
            self.params = None
            self.pos = [None] * self.n_gates
        elif kind == "rigid":
            self.params = np.asarray(params, dtype=np.float64)
            self.n_gates = self.params.shape[0]
            self.pos = [warp.rigid_positions(n, *self.params[i]) for i in range(self.n_gates)]
        elif kind == "field":
            self.params = np.asarray(params, dtype=np.float64)
            self.n_gates = self.params.shape[0]
            self.pos = [warp.field_positions(self.params[i]) for i in range(self.n_gates)]
        else:
            raise ValueError(kind)

    def D(self, i, x):
        if self.pos[i] is None:
            return np.asarray(x, dtype=np.float64).copy()
        return warp.warp(x, *self.pos[i])

    def Dt(self, i, b):
        if self.pos[i] is None:
            return np.asarray(b, dtype=np.float64).copy()
        return warp.warp_adjoint(b, *self.pos[i])

    def project(self, x):
        if self.matrix is not None:
            v = self.matrix @ np.asarray(x, dtype=np.float64).ravel()
            return v.reshape(self.n_angles, self.n_det)
        return projector.forward(x, self.n_angles, self.n_det)

    def backproject(self, y):
        if self.matrix is not None:
            v = self.matrix.T @ np.asarray(y, dtype=np.float64).ravel()
            return v.reshape(self.n, self.n)
        return projector.adjoint(y, self.n)

    def A(self, i, x):
        """A_i x = A D_i x."""
        return self.project(self.D(i, x))

    def At(self, i, y):
        """A_i^* y = D_i^T A^T y."""
        return self.Dt(i, self.backproject(y))
