"""FP64 CPU oracle for motion-compensated SPDHG/PDHG reconstruction.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
HIP library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
shares no code, tables or constants with it.

Everything is float64 NumPy, written from the paper's definitions:

* `projector` - the ray transform A (Section II-A, with the Joseph
  discretisation of a 2D parallel-beam geometry read from Section III) and its
  exact transpose, built as a scatter of the same weights;
* `warp`      - the displacement operator D_i (Section II-A) as a bilinear
  pull-back with zero padding, rigid or displacement-field, and its transpose;
* `spdhg`     - the proximal maps, Algorithm 1 (SPDHG; PDHG as the case p_i=1,
  S = all gates), the step sizes behind Theorem 1, the rate l(kappa, n),
  power iteration for the operator norms, the saddle point as a linear solve,
  the objective, the duality gap and the distance plotted in Fig. 1;
* `grad`      - the gradient of a loss through unrolled SPDHG iterations with
  respect to the starting image and the motion parameters (transposed iteration
  map);
* `subsets`   - SPDHG over gates x angle subsets;
* `registration` - rigid, affine and dense displacement-field registration of
  a gate's image to the reference (the preliminary step of Section I; the
  readings are stated there).

Where the paper is silent or garbled, the readings are listed in the design
notes: step (i) uses the extrapolated z-bar, step (iii) extrapolates from z,
f_i(u) = |u - d_i|^2 / N and g(x) = alpha |x|^2.
"""
from . import projector, warp, spdhg, grad, subsets, registration  # noqa: F401
from .operators import GatedOperators  # noqa: F401
