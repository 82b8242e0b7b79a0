"""mcr_project_noalloc (the projection that allocates nothing) against
mcr_project of a float32 handle, through the C ABI: several calls in a row on
one GPU, each smaller than the one before, so that what an earlier call left
in the shared scratch array cannot leak into a later result."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import F32_OP, need_gpu, rel

pytestmark = pytest.mark.gpu

# (n, n_angles, n_det): a large case, a smaller one, then a ragged odd one
CASES = [(512, 360, 730), (256, 180, 366), (97, 75, 141)]


def _reference(n, na, nd, x, variant):
    from paper_2410_10503_amd import Handle
    h = Handle(n, na, nd, ["identity"], dtype=torch.float32)
    if variant is not None:
        h.set_variant(*variant)
    out = h.project(x)
    torch.cuda.synchronize()
    h.close()
    return out.double().cpu().numpy()


def test_noalloc_projection_matches_handle_projection():
    need_gpu()
    from paper_2410_10503_amd import project_noalloc
    for call, (n, na, nd) in enumerate(CASES):
        print(f"no-alloc projection call {call}: n={n} n_angles={na} n_det={nd}", flush=True)
        x = torch.from_numpy(synth.random_image(n, 40 + call)).cuda()
        out = torch.full((na, nd), float("nan"), dtype=torch.float32, device="cuda")
        project_noalloc(x, na, nd, out)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        assert np.all(np.isfinite(got))
        # the handle on the same kernel (forward variant 0): the same weights
        # summed in the same order
        same = _reference(n, na, nd, x, (0, 8, 6))
        assert rel(got, same) <= F32_OP
        assert np.max(np.abs(got - same)) <= 1e-6 * np.max(np.abs(same))
        # the handle's default projector (another summation order)
        ref = _reference(n, na, nd, x, None)
        assert rel(got, ref) <= F32_OP
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
        print(f"  rel L2 vs handle (variant 0) {rel(got, same):.2e}, vs default {rel(got, ref):.2e}, "
              f"bitwise equal to variant 0: {bool(np.array_equal(got, same))}", flush=True)


def test_noalloc_projection_rejects_sizes_beyond_its_scratch():
    need_gpu()
    from paper_2410_10503_amd import McrError, project_noalloc
    x = torch.zeros((1100, 1100), dtype=torch.float32, device="cuda")
    out = torch.zeros((10, 1600), dtype=torch.float32, device="cuda")
    with pytest.raises(McrError, match="MCR_ERR_ARG"):
        project_noalloc(x, 10, 1600, out)
