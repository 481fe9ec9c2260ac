"""Signed distance of a voxel image on the GPU (exact distance transform) against the
oracle, through the C ABI: the squared distances are integers, so the FP32 results are
bit-identical."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _check(rd, oracle_mod, img, dx=1.0):
    got = rd.sdf_from_image(np.ascontiguousarray(img, dtype=np.uint8), dx).cpu().numpy()
    want = oracle_mod.signed_distance(img, dx)
    bad = np.argwhere(got != want)
    assert len(bad) == 0, (img.shape, bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])


@pytest.mark.parametrize("seed,porosity", [(1, 0.3), (2, 0.6), (3, 0.9)])
def test_random_volumes(rd, oracle_mod, seed, porosity):
    img, _ = W.boolean_spheres(48, porosity, 2.0, 5.0, seed=seed)
    _check(rd, oracle_mod, np.ascontiguousarray(img[:37, :41, :29]), dx=0.37)


def test_tiny_and_degenerate(rd, oracle_mod):
    for seed in range(8):
        _check(rd, oracle_mod, W.random_tiny_geometry(seed))
    _check(rd, oracle_mod, np.ones((5, 6, 7), np.uint8))
    _check(rd, oracle_mod, np.zeros((5, 6, 7), np.uint8))
    one = np.zeros((9, 10, 11), np.uint8)
    one[4, 5, 6] = 1
    _check(rd, oracle_mod, one)
    _check(rd, oracle_mod, 1 - one)
    rng = np.random.default_rng(4)
    for shape in [(1, 1, 40), (1, 40, 1), (40, 1, 1), (1, 1, 1), (2, 1, 3)]:
        _check(rd, oracle_mod, (rng.random(shape) < 0.5).astype(np.uint8), dx=2.0)


def test_packing_and_ball(rd, oracle_mod):
    img, _ = W.workload_geometry("spheres64")
    _check(rd, oracle_mod, img)
    ball, _ = W.single_sphere(70, (34.5, 35.2, 33.8), 21.3)
    _check(rd, oracle_mod, ball, dx=1.0 / 70)


def test_feeds_geometry_and_diffusivity(rd, oracle_mod):
    """The GPU SDF passes the geometry's sign check and sets the same factor as the
    oracle's SDF."""
    img, _ = W.boolean_spheres(40, 0.5, 2.0, 4.0, seed=8)
    sdf = rd.sdf_from_image(img, 1.0)
    g = rd.Geometry(img, sdf.cpu().numpy(), 1.0, 8)
    outs = []
    for phi in (sdf, oracle_mod.signed_distance(img, 1.0)):
        s = rd.Sim(g, "fp32")
        s.add_species(1.0)
        s.set_dirichlet(0, 0, 1.0)
        s.bind(features=rd.RD_WS_DIFFUSIVITY)
        s.set_diffusivity_sdf(phi, 0.1, 0.9, -6.0, 4.0)
        s.step(0.1, 50)
        outs.append(s.get_field(0).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_errors(rd):
    with pytest.raises(rd.RDError):
        rd.sdf_from_image(np.ones((4, 4, 4), np.uint8), 0.0)
