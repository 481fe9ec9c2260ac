"""Pins of the oracle's signed distance of a voxel image (eq. SDF of section
"Level-set method for image-based geometry reconstruction"): brute force over all
voxel pairs on tiny volumes, the one-phase cases, and first-order convergence to the
exact distance of a ball (the paper's SDF converges at first order as well)."""
import math

import numpy as np
import pytest

import workloads as W


def _brute(img, dx):
    img = img != 0
    pts = np.argwhere(np.ones_like(img)).astype(np.float64)
    flat = img.ravel()
    act, ina = pts[flat], pts[~flat]
    diag = math.sqrt(float(np.sum(np.square(img.shape))))
    out = np.empty(len(pts))
    for i, p in enumerate(pts):
        other = ina if flat[i] else act
        d = diag if len(other) == 0 else math.sqrt(((other - p) ** 2).sum(axis=1).min()) - 0.5
        out[i] = d if flat[i] else -d
    return (out * dx).reshape(img.shape)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force(oracle_mod, seed):
    img = W.random_tiny_geometry(seed, shape=(6, 7, 9))
    got = oracle_mod.signed_distance(img, 0.7)
    np.testing.assert_allclose(got, _brute(img, 0.7), rtol=1e-6, atol=1e-6)
    assert np.all((got > 0) == (img != 0))


def test_one_phase(oracle_mod):
    for v in (0, 1):
        img = np.full((3, 4, 5), v, np.uint8)
        got = oracle_mod.signed_distance(img, 2.0)
        want = math.sqrt(9 + 16 + 25) * 2.0 * (1 if v else -1)
        assert np.all(got == np.float32(want))


def test_ball_first_order(oracle_mod):
    errs = []
    for n in (24, 48, 96):
        h = 2.0 / n  # box [-1, 1]^3 sampled at voxel centres, ball of radius 0.6
        x = (np.arange(n) + 0.5) * h - 1.0
        z, y, xx = np.meshgrid(x, x, x, indexing="ij")
        exact = 0.6 - np.sqrt(xx ** 2 + y ** 2 + z ** 2)
        img = (exact > 0).astype(np.uint8)
        got = oracle_mod.signed_distance(img, h)
        near = np.abs(exact) < 0.3
        errs.append(np.max(np.abs(got[near] - exact[near])))
    o1, o2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert errs[2] < 0.03
    assert 0.7 < o1 < 1.6 and 0.7 < o2 < 1.6, (errs, o1, o2)
