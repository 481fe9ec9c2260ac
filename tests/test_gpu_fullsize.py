"""The headline workload at its full size (512^3 soil-like volume, two species, 8^3
blocks, the launch configuration bench.py times after autotuning):

* 10 steps compared element by element with the FP64 oracle on the whole volume;
* the full 10 000 steps, then one more step checked against the discrete balance
  M' - M = dt (inflow - uptake + reactions) of each species in FP64, a property that
  holds at any size.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd

    w = W.workload("soil512")
    img = W.gaussian_random_field_volume(512, 12.0, 0.3, seed=w.seed)
    g = rd.Geometry(img, None, w.dx, 8)
    s = rd.Sim(g, "fp32")
    for d in w.species_D:
        s.add_species(d)
    for (a, b, k) in w.reactions:
        s.add_reaction(a, b, k)
    for sp, k in w.robin.items():
        s.set_robin(sp, k)
    for (sp, f), v in w.dirichlet.items():
        s.set_dirichlet(sp, f, v)
    s.bind()
    s.autotune(w.dt, 100)
    return rd, w, img, g, s


def test_full_size_first_steps_vs_oracle(setup, oracle_mod):
    rd, w, img, g, s = setup
    s.step(w.dt, 10)
    got = np.stack([s.get_field(i).cpu().numpy() for i in range(2)]).astype(np.float64)
    prob = oracle_mod.Problem(img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                              reactions=w.reactions)
    ref = prob.run(prob.initial(), w.dt, 10)
    act = img != 0
    for sp in range(2):
        err = rel_l2(got[sp], ref[sp], act)
        print(f"512^3 species {sp}, 10 steps: rel L2 {err:.3e}")
        assert err < 1e-6
    assert np.all(got[:, ~act] == 0)


def test_full_size_balance_after_full_run(setup):
    rd, w, img, g, s = setup
    s.step(w.dt, w.steps - s.steps_taken())
    assert s.steps_taken() == w.steps
    before = [s.balance(sp) for sp in range(2)]
    s.step(w.dt, 1)
    after = [s.balance(sp) for sp in range(2)]
    for sp in range(2):
        b0, b1 = before[sp], after[sp]
        pred = w.dt * (b0["inflow"].sum() - b0["uptake"] + b0["react"])
        got = b1["mass"] - b0["mass"]
        scale = w.dt * max(abs(b0["inflow"].sum()), abs(b0["uptake"]), abs(b0["react"]))
        print(f"species {sp}: dM {got:.6f} predicted {pred:.6f} (scale {scale:.3f})")
        assert abs(got - pred) <= 2e-3 * scale
    # the front has moved into the volume and B has been produced
    assert before[0]["mass"] > 0 and before[1]["mass"] > 0
