"""The inhomogeneous-diffusion form at its full size (512^3 soil-like volume, two species,
8^3 blocks, the smooth D(phi) factor from the GPU signed distance, the column kernel the
bench times), checked through properties that hold at any size:

* one step satisfies the discrete balance M' - M = dt (inflow - uptake + reactions) of
  each species in FP64 (inflow with the mean face coefficient);
* the column kernel and the one-thread-per-slot kernel give the same bits.
Element-by-element parity with the oracle runs at small sizes (test_gpu_diffusivity).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

PARS = (0.1, 0.9, -6.0, 4.0)


@pytest.fixture(scope="module")
def setup():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd

    w = W.workload("soil512")
    img = W.gaussian_random_field_volume(512, 12.0, 0.3, seed=w.seed)
    g = rd.Geometry(img, None, w.dx, 8)
    phi = rd.sdf_from_image(img, w.dx)
    return rd, w, img, g, phi


def _sim(rd, w, g, phi, kernel):
    s = rd.Sim(g, "fp32")
    for d in w.species_D:
        s.add_species(d)
    for (a, b, k) in w.reactions:
        s.add_reaction(a, b, k)
    for sp, k in w.robin.items():
        s.set_robin(sp, k)
    for (sp, f), v in w.dirichlet.items():
        s.set_dirichlet(sp, f, v)
    s.set_kernel(kernel)
    s.bind(features=rd.RD_WS_DIFFUSIVITY)
    s.set_diffusivity_sdf(phi, *PARS)
    return s


def test_full_size_balance(setup):
    rd, w, img, g, phi = setup
    s = _sim(rd, w, g, phi, "column_xch")
    s.step(w.dt, 500)
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
    assert before[0]["mass"] > 0 and before[1]["mass"] > 0


def test_full_size_kernels_agree(setup):
    rd, w, img, g, phi = setup
    outs = []
    for kernel in ("column_xch", "column", "block"):
        s = _sim(rd, w, g, phi, kernel)
        s.step(w.dt, 40)
        outs.append([s.get_field(sp).cpu().numpy() for sp in range(2)])
        del s
    for o in outs[1:]:
        for sp in range(2):
            assert np.array_equal(outs[0][sp], o[sp])
