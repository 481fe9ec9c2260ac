"""The compact field layout (only the active voxels of each stored 8^3 block are kept)
against the block layout: the same kernels' arithmetic on the same values, so every
field, balance term, plane flux and region mass must be bitwise equal; and the compact
run against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _sim(rd, img, layout, storage, S, kernel="column", graph=True, xcd=True, sround=False):
    g = rd.Geometry(img, None, 1.0, 8)
    s = rd.Sim(g, storage)
    Ds = [1.0, 0.4, 0.7, 0.25][:S]
    for d in Ds:
        s.add_species(d)
    if S >= 2:
        s.add_reaction(0, 1, 0.01)
        s.set_robin(1, 0.05)
    if S >= 3:
        s.add_reaction(2, -1, 0.02)
        s.set_dirichlet(2, 3, 0.5)
        s.set_dirichlet(2, 4, 0.25)
    if S >= 4:
        s.add_reaction(1, 3, 0.03)
    s.set_dirichlet(0, 0, 1.0)
    s.set_launch(16, graph, xcd)
    s.set_layout(layout)
    s.set_kernel(kernel)
    if sround:
        s.set_rounding(1, seed=99)
    s.bind()
    return g, s


def _state(s, S):
    f = np.stack([s.get_field(i).cpu().numpy() for i in range(S)])
    bal = [s.balance(i) for i in range(S)]
    return f, bal


def _ragged(seed, shape=(45, 38, 51), p=0.45):
    img, _ = W.boolean_spheres(shape, p, 2.0, 5.0, seed=seed)
    img[:, :, 0] |= (np.arange(shape[1])[None, :] % 3 == 0).astype(np.uint8)  # inlet voxels
    return np.ascontiguousarray(img)


@pytest.mark.parametrize("storage,sround", [("fp32", False), ("fp32", True), ("bf16", False),
                                            ("bf16", True), ("fp16", True)])
@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_compact_equals_blocks(rd, storage, sround, S):
    img = _ragged(20 + S)
    runs = {}
    for layout, kernels in (("blocks", ("column", "column_xch")),
                            ("compact", ("column", "column_xch", "column_lanes"))):
        for kernel in kernels:
            g, s = _sim(rd, img, layout, storage, S, kernel=kernel, sround=sround)
            s.step(0.1, 37)
            runs[(layout, kernel)] = _state(s, S)
    ref_f, ref_b = runs[("blocks", "column")]
    for key, (f, b) in runs.items():
        np.testing.assert_array_equal(f, ref_f, err_msg=str(key))
        for i in range(S):
            for k in ("mass", "uptake", "react"):
                assert b[i][k] == ref_b[i][k], (key, i, k)
            np.testing.assert_array_equal(b[i]["inflow"], ref_b[i]["inflow"])


def test_compact_direct_launches_and_fluxes(rd):
    img = _ragged(7, shape=(33, 41, 40))
    out = {}
    for layout, kernel in (("blocks", "column"), ("compact", "column"), ("compact", "column_lanes")):
        g, s = _sim(rd, img, layout, "fp32", 2, kernel=kernel, graph=False, xcd=False)
        s.step(0.1, 23)
        fl = [s.plane_flux(sp, ax, i0) for sp in range(2) for ax in range(3) for i0 in (0, 7, 8, 15, 30)]
        rm = [s.region_mass(sp, (3, 17, 5, 29, 8, 9)) for sp in range(2)]
        rm.append(s.region_mass(0, (0, 40, 0, 41, 0, 33)))
        out[(layout, kernel)] = (_state(s, 2)[0], fl, rm)
    ref = out[("blocks", "column")]
    for key, val in out.items():
        np.testing.assert_array_equal(val[0], ref[0], err_msg=str(key))
        assert val[1] == ref[1] and val[2] == ref[2], key


def test_compact_set_field_roundtrip_and_oracle(rd, oracle_mod):
    import torch

    img = _ragged(9, shape=(40, 36, 44))
    rng = np.random.default_rng(5)
    u0 = rng.random(img.shape).astype(np.float32)
    g, s = _sim(rd, img, "compact", "fp32", 2)
    for sp in range(2):
        s.set_field(sp, torch.from_numpy(u0 * (sp + 1)).to("cuda"))
    back = np.stack([s.get_field(sp).cpu().numpy() for sp in range(2)])
    want = np.stack([np.where(img != 0, u0 * (sp + 1), 0) for sp in range(2)])
    want[0][:, :, 0][img[:, :, 0] != 0] = 1.0  # the held inlet value
    np.testing.assert_array_equal(back, want)
    s.step(0.1, 200)
    got = np.stack([s.get_field(sp).cpu().numpy() for sp in range(2)]).astype(np.float64)
    prob = oracle_mod.Problem(img, [1.0, 0.4], robin={1: 0.05}, dirichlet={(0, 0): 1.0},
                              reactions=[(0, 1, 0.01)])
    ref = prob.run(want.astype(np.float64), 0.1, 200)
    for sp in range(2):
        err = rel_l2(got[sp], ref[sp], img != 0)
        print(f"compact, species {sp}, 200 steps from a random field: rel L2 {err:.2e}")
        assert err < 1e-6


def test_compact_soil_full_size_equals_blocks(rd):
    """The benchmark's volume and launch: the autotuned compact run gives the block
    layout's bits after 100 steps."""
    w = W.workload("soil512")
    img, _ = W.workload_geometry("soil512")
    res = {}
    for layout in ("blocks", "compact"):
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
        s.set_layout(layout)
        s.bind()
        s.autotune(w.dt, 40)
        s.step(w.dt, 100)
        res[layout] = [s.get_field(i).cpu().numpy() for i in range(2)] + [s.balance(0)["mass"]]
        print(layout, s.get_launch())
        del s
    for i in range(2):
        np.testing.assert_array_equal(res["compact"][i], res["blocks"][i])
    assert res["compact"][2] == res["blocks"][2]
