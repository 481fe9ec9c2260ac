"""Several steps per cooperative launch (rd_sim_set_fused_steps) against one launch per step.

A fused launch runs the column kernel's per-block work for each step in turn, with a grid
barrier between the steps, the buffers swapped and each step's rounding key: the fields
must equal those of single-step launches bit for bit, for step counts that are not a
multiple of the steps per launch, and for several geometries stepped together."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

D = [1.0, 0.4]
REACT = [(0, 1, 0.02)]
ROBIN = {1: 0.05}
DIR = {(0, 0): 1.0}
DT = 0.1


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _sim(rd, g, storage, kernel, sround, fused):
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
        s.set_rounding(1, seed=9)
    s.set_launch(16, True, True)
    s.set_kernel(kernel, 8)
    s.set_fused_steps(fused)
    s.bind()
    return s


def _images():
    rng = np.random.default_rng(21)
    return {"spheres64": W.workload_geometry("spheres64")[0],
            "ragged": (rng.random((37, 29, 45)) < 0.55).astype(np.uint8)}


@pytest.mark.parametrize("storage,sround,kernel", [
    ("fp32", False, "column_xch"), ("fp32", True, "column_xch"), ("fp32", True, "column"),
    ("bf16", True, "column"), ("fp16", True, "column_xch")])
def test_fused_equals_single_step_launches(rd, storage, sround, kernel):
    for name, img in _images().items():
        g = rd.Geometry(img, None, 1.0, 8)
        ref = _sim(rd, g, storage, kernel, sround, 1)
        ref.step(DT, 50)
        for fused in (2, 7, 16):
            s = _sim(rd, g, storage, kernel, sround, fused)
            assert s.get_fused_steps() == fused
            s.step(DT, 20)
            s.step(DT, 30)  # two calls: the counter and the buffer parity carry over
            assert s.steps_taken() == 50
            for sp in range(len(D)):
                a, b = s.get_field(sp), ref.get_field(sp)
                assert bool((a == b).all()), f"{name}: {fused} steps per launch differ (species {sp})"
            assert s.balance(1)["mass"] == ref.balance(1)["mass"]


def test_fused_concatenated_parts_equal_single_runs(rd):
    imgs = list(_images().values())
    gs = [rd.Geometry(img, None, 1.0, 8) for img in imgs]
    cat = rd.Geometry.concat(gs)
    sc = _sim(rd, cat, "fp32", "column_xch", True, 16)
    sc.step(DT, 40)
    for i, g in enumerate(gs):
        s1 = _sim(rd, g, "fp32", "column_xch", True, 1)
        s1.step(DT, 40)
        for sp in range(len(D)):
            assert bool((sc.get_part_field(sp, i) == s1.get_field(sp)).all())
