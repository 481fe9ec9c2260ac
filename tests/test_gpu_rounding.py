"""Stochastic rounding against its definition, on a field where the exact result of a step
sits a known fraction of the storage spacing between two stored values.

A uniform all-active box of c = 1.5 with first-order decay only (the Laplacian of a uniform
field is exactly 0): one step gives c (1 - beta) with beta = dt k a power of two, so the
FP32 result 1.5 - 1.5 beta is exact and lies the fraction f = 1.5 beta / spacing below 1.5
on the storage grid (spacing 2^-23 for FP32, 2^-7 for BF16, 2^-10 for FP16 in [1, 2)).
Stochastic rounding must then store 1.5 - spacing with probability f and 1.5 otherwise:
over N voxels the fraction rounded down is f within a few standard errors
sqrt(f (1 - f) / N), every voxel holds one of the two values, and the choices of x-adjacent
voxels and of the same voxel in two seeds are independent (pair fraction f^2).  FP32
rounds through the dither (u - 1/2) ulp(c) added to the increment; BF16 and FP16 round
at the store."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 64


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


# storage: (spacing of the storage type in [1, 2), dt, decay rate) with beta = dt * rate
CASES = {"fp32": (2.0 ** -23, 2.0 ** -6, 2.0 ** -20),   # beta 2^-26: f = 0.1875
         "bf16": (2.0 ** -7, 2.0 ** -6, 2.0 ** -3),     # beta 2^-9:  f = 0.375
         "fp16": (2.0 ** -10, 2.0 ** -6, 2.0 ** -6)}    # beta 2^-12: f = 0.375


def _one_step(rd, storage, seed, kernel, B):
    import torch

    spacing, dt, rate = CASES[storage]
    img = np.ones((N, N, N), dtype=np.uint8)
    g = rd.Geometry(img, None, 1.0, B)
    s = rd.Sim(g, storage)
    s.add_species(1.0)
    s.add_reaction(0, -1, rate)
    s.set_rounding(1, seed=seed)
    if B == 8:
        s.set_kernel(kernel, 8)
    s.bind()
    s.set_field(0, np.full((N, N, N), 1.5, dtype=np.float32))
    s.step(dt, 1)
    out = s.get_field(0).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    return out, spacing, 1.5 * dt * rate / spacing


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("kernel,B", [("column_xch", 8), ("block", 8), ("block", 4)])
def test_stochastic_rounding_probabilities(rd, storage, kernel, B):
    a, spacing, f = _one_step(rd, storage, 3, kernel, B)
    lo = 1.5 - spacing
    assert np.all((a == 1.5) | (a == lo)), "values other than the two neighbours of the exact result"
    down = a == lo
    n = down.size
    se = np.sqrt(f * (1 - f) / n)
    frac = down.mean()
    assert abs(frac - f) < 5 * se, f"fraction rounded down {frac:.5f}, expected {f} +- {se:.5f}"
    # independence of neighbours along x (overlapping pairs share a voxel: the variance of
    # the pair fraction gains 2 (f^3 - f^4) per pair) and between seeds
    m = down[:, :, 1:].size
    pair = (down[:, :, 1:] & down[:, :, :-1]).mean()
    assert abs(pair - f * f) < 6 * np.sqrt((f * f * (1 - f * f) + 2 * (f ** 3 - f ** 4)) / m)
    b, _, _ = _one_step(rd, storage, 4, kernel, B)
    both = (down & (b == lo)).mean()
    assert abs(both - f * f) < 5 * np.sqrt(f * f * (1 - f * f) / n)
    assert not np.array_equal(down, b == lo)
