"""Several geometries stepped together (rd_geometry_concat) against each stepped alone.

Each part of a concatenated geometry takes the same per-voxel operations in the same order
as when it is stepped on its own (its block neighbours, box faces and stochastic-rounding
bits are its own), so its field must equal the single run's bit for bit.  The per-part
balance sums the same FP64 terms over the same blocks, grouped into other rows, so it
agrees to rounding.  Part 0 is also compared with the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu

D = [1.0, 0.4]
REACT = [(0, 1, 0.02)]
ROBIN = {1: 0.05}
DIR = {(0, 0): 1.0}  # species A held at 1 on each part's own x = 0 face
DT = 0.1


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _images():
    rng = np.random.default_rng(11)
    shapes = [(21, 18, 27), (9, 33, 12), (17, 17, 17), (3, 5, 7), (30, 14, 19)]
    imgs = [(rng.random(s) < p).astype(np.uint8) for s, p in zip(shapes, (0.6, 0.5, 0.7, 0.9, 0.55))]
    imgs[2][:, :, :] = 0  # a part without active voxels: no blocks
    return imgs


def _setup(rd, g, storage, kernel, sround, B):
    s = rd.Sim(g, storage)
    for d in D:
        s.add_species(d)
    for a, b, k in REACT:
        s.add_reaction(a, b, k)
    for sp, k in ROBIN.items():
        s.set_robin(sp, k)
    for (sp, f), v in DIR.items():
        s.set_dirichlet(sp, f, v)
    if sround:
        s.set_rounding(1, seed=77)
    s.set_launch(16, True, True)
    if B == 8:
        s.set_kernel(kernel, 8)
    s.bind()
    return s


@pytest.mark.parametrize("B,storage,sround,kernel", [
    (8, "fp32", False, "column_xch"), (8, "fp32", True, "column_xch"), (8, "fp32", False, "block"),
    (8, "bf16", True, "column"), (4, "fp32", True, "block"), (4, "fp16", True, "block")])
def test_parts_equal_single_runs(rd, B, storage, sround, kernel):
    imgs = _images()
    singles = [rd.Geometry(img, None, 1.0, B) for img in imgs]
    cat = rd.Geometry.concat(singles)
    parts = cat.parts()
    assert len(parts) == len(imgs)
    assert sum(p["n_blocks"] for p in parts) == cat.stats()["n_blocks"]
    sc = _setup(rd, cat, storage, kernel, sround, B)
    # a random initial field: the parts' boxes one after another in one dense array
    rng = np.random.default_rng(5)
    inits = [[rng.random(img.shape).astype(np.float32) for _ in D] for img in imgs]
    for sp in range(len(D)):
        sc.set_field(sp, np.concatenate([ini[sp].ravel() for ini in inits]))
    steps = 150
    sc.step(DT, steps)
    tot = [sc.balance(sp) for sp in range(len(D))]
    for i, (g, img) in enumerate(zip(singles, imgs)):
        if not img.any():  # no blocks: nothing stored, the part reads back as zeros
            for sp in range(len(D)):
                assert not sc.get_part_field(sp, i).cpu().numpy().any()
                assert sc.balance(sp, part=i)["mass"] == 0.0
            continue
        s1 = _setup(rd, g, storage, kernel, sround, B)
        for sp in range(len(D)):
            s1.set_field(sp, inits[i][sp])
        s1.step(DT, steps)
        for sp in range(len(D)):
            a = sc.get_part_field(sp, i).cpu().numpy()
            b = s1.get_field(sp).cpu().numpy()
            assert np.array_equal(a, b), f"part {i} species {sp} differs from its single run"
            bp, b1 = sc.balance(sp, part=i), s1.balance(sp)
            assert bp["mass"] == pytest.approx(b1["mass"], rel=1e-12, abs=1e-12)
            assert bp["uptake"] == pytest.approx(b1["uptake"], rel=1e-12, abs=1e-12)
            assert bp["react"] == pytest.approx(b1["react"], rel=1e-12, abs=1e-12)
            np.testing.assert_allclose(bp["inflow"], b1["inflow"], rtol=1e-12, atol=1e-12)
    for sp in range(len(D)):
        msum = sum(sc.balance(sp, part=i)["mass"] for i in range(len(imgs)))
        assert msum == pytest.approx(tot[sp]["mass"], rel=1e-12)


def test_part_vs_oracle(rd, oracle_mod):
    imgs = _images()
    singles = [rd.Geometry(img, None, 1.0, 8) for img in imgs]
    cat = rd.Geometry.concat(singles)
    sc = _setup(rd, cat, "fp32", "column_xch", False, 8)
    steps = 300
    sc.step(DT, steps)
    for i in (0, 4):
        prob = oracle_mod.Problem(imgs[i], D, robin=ROBIN, dirichlet=DIR, reactions=REACT)
        ref = prob.run(prob.initial(), DT, steps)
        act = imgs[i] != 0
        for sp in range(len(D)):
            got = sc.get_part_field(sp, i).cpu().numpy().astype(np.float64)
            assert rel_l2(got, ref[sp], act) < 1e-5


def test_single_box_calls_refused(rd):
    imgs = _images()
    cat = rd.Geometry.concat([rd.Geometry(img, None, 1.0, 8) for img in imgs])
    s = rd.Sim(cat, "fp32")
    s.add_species(1.0)
    s.bind(features=rd.RD_WS_SOLVER)
    with pytest.raises(rd.RDError, match="STATE"):
        s.steady_state(0, 1e-6, 100)
    with pytest.raises(rd.RDError, match="STATE"):
        s.plane_flux(0, 0, 1)
    with pytest.raises(rd.RDError, match="ARG"):
        s.balance(0, part=len(imgs))
