"""The allocation-free signed-distance entry point (rd_sdf_from_image_static, fixed
per-GPU scratch) against the one with a caller scratch (rd_sdf_from_image): the same
kernels, so the same bits, on two calls in a row, the second on a smaller volume."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_static_scratch_matches_caller_scratch():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd

    shapes = [(144, 140, 136), (40, 52, 33)]
    for i, shape in enumerate(shapes):
        img, _ = W.boolean_spheres(shape, 0.5, 3.0, 9.0, seed=60 + i)
        dimg = torch.from_numpy(img).to("cuda")
        ref = rd.sdf_from_image(dimg, 0.5)
        out = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
        rd.sdf_from_image_static(dimg, out, 0.5)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        print(f"call {i}: shape {shape}, {int(img.sum())} active voxels, "
              f"max |diff| {float(np.max(np.abs(a - b))):.3g}")
        np.testing.assert_array_equal(a, b)
        assert np.all((b > 0) == (img != 0))


def test_static_scratch_rejects_large_volume():
    import torch

    from paper_2304_11165_amd import rd

    img = torch.zeros((160, 160, 160), dtype=torch.uint8, device="cuda")
    out = torch.empty((160, 160, 160), dtype=torch.float32, device="cuda")
    with pytest.raises(rd.RDError):
        rd.sdf_from_image_static(img, out)
