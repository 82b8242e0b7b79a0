// Device code of the rigid registration (the preliminary step of Section I:
// the displacement maps from the reference state to each gate): the residual
// of the warped reference against the gate's image, written into the padded
// layout that the motion-gradient kernel reads. The warp, the reductions and
// the motion gradient are the library's own kernels.
#pragma once

#include "mcr_kernels.h"

namespace mcr {

// rP = wP - target on the image (the zero border of rP is left as it is).
// grid (ceil(n/16), ceil(n/16)), block (16, 16)
template <typename T>
__global__ __launch_bounds__(256) void k_residual_padded(int n, int pitch, const T* __restrict__ wP,
                                                         const T* __restrict__ target, T* __restrict__ rP) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c < n && r < n) {
    const long q = (long)(r + kPad) * pitch + c + kPad;
    rP[q] = wP[q] - target[(long)r * n + c];
  }
}

}  // namespace mcr
