"""Inhomogeneous diffusion on the GPU (per-voxel diffusivity factor, mean coefficient
on each face) against the FP64 oracle, through the C ABI.

Tolerance: relative L2 over active voxels <= 1e-5 for FP32 storage, as for the
homogeneous step (FP32 rounding of ~1e-7 per step, damped by diffusion).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import fields, make_gpu, rel_l2, round_to_storage

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _problem(seed=31, shape=(19, 23, 29)):
    """Ragged box (no edge a multiple of 4 or 8), overlapping spheres removed, random
    factor in [0.2, 1.5]."""
    img, _ = W.boolean_spheres(max(shape), 0.6, 2.0, 4.0, seed=seed)
    img = np.ascontiguousarray(img[:shape[0], :shape[1], :shape[2]])
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.2, 1.5, size=img.shape)
    return img, eps


def _run(rd, oracle_mod, img, eps, D, dt, n, B, kernel, storage="fp32", robin=None,
         dirichlet=None, reactions=None, init=None, graph=True, sround=False):
    g, s = make_gpu(rd, img, D, 1.0, robin, dirichlet, reactions, storage, B, graph=graph,
                    kernel=kernel, features=rd.RD_WS_DIFFUSIVITY)
    if sround:
        s.set_rounding(True, 7)
    e32 = eps.astype(np.float32)
    s.set_diffusivity(e32)
    prob = oracle_mod.Problem(img, D, robin=robin, dirichlet=dirichlet, reactions=reactions,
                              eps=e32.astype(np.float64))
    c0 = prob.initial()
    if init is not None:
        c0 = prob.apply_dirichlet(round_to_storage(init, storage))
        for sp in range(len(D)):
            s.set_field(sp, c0[sp].astype(np.float32))
    s.step(dt, n)
    return fields(s, len(D)), prob.run(c0, dt, n), prob, s


CASE = dict(D=[1.0, 0.4], robin={0: 0.05}, dirichlet={(0, 0): 1.0, (1, 5): 0.25},
            reactions=[(0, 1, 0.03), (1, -1, 0.01)])


@pytest.mark.parametrize("B,kernel", [(8, "column"), (8, "block"), (4, "block")])
def test_parity_with_oracle(rd, oracle_mod, B, kernel):
    img, eps = _problem()
    rng = np.random.default_rng(5)
    init = rng.uniform(0, 1, (2,) + img.shape)
    dt = 0.9 / (12 * 1.5 + 0.03 + 6 * 0.05)  # below the bound with max(e) = 1.5
    got, ref, prob, s = _run(rd, oracle_mod, img, eps, CASE["D"], dt, 60, B, kernel,
                             robin=CASE["robin"], dirichlet=CASE["dirichlet"],
                             reactions=CASE["reactions"], init=init)
    act = img != 0
    for sp in range(2):
        err = rel_l2(got[sp], ref[sp], act)
        print(f"B={B} {kernel} species {sp}: rel L2 {err:.3e}")
        assert err < TOL
        assert np.all(got[sp][~act] == 0)
    # balance terms of the GPU field against the oracle's on the same field
    for sp in range(2):
        b = s.balance(sp)
        m, infl, up, re = prob.balance(got, sp)
        assert b["mass"] == pytest.approx(m, rel=1e-10, abs=1e-12)
        np.testing.assert_allclose(b["inflow"], infl, rtol=1e-9, atol=1e-12)
        assert b["uptake"] == pytest.approx(up, rel=1e-10, abs=1e-12)
        assert b["react"] == pytest.approx(re, rel=1e-10, abs=1e-12)
    assert s.balance(0)["inflow"][0] != 0.0
    # plane fluxes with the mean face coefficient, on and off block boundaries
    for axis, n in ((0, img.shape[2]), (1, img.shape[1]), (2, img.shape[0])):
        for i0 in (0, 3, 7, 8, 15, n - 2):
            for sp in range(2):
                want = prob.plane_flux(got[sp], CASE["D"][sp], axis, i0)
                assert s.plane_flux(sp, axis, i0) == pytest.approx(want, rel=1e-10, abs=1e-13), \
                    (B, axis, i0, sp)


@pytest.mark.parametrize("storage,sround", [("fp32", False), ("bf16", True), ("fp16", False)])
def test_kernels_agree_bitwise(rd, oracle_mod, storage, sround):
    """B = 8 column kernel == with the x-face exchange == one thread per slot, graph replay ==
    direct launches."""
    img, eps = _problem(seed=9, shape=(27, 21, 34))
    rng = np.random.default_rng(9)
    init = rng.uniform(0, 1, (2,) + img.shape)
    dt = 0.05
    outs = []
    for kernel, graph in (("column", True), ("block", False), ("column", False), ("column_xch", True),
                          ("column_xch", False)):
        got, _, _, _ = _run(rd, oracle_mod, img, eps, CASE["D"], dt, 70, 8, kernel, storage=storage,
                            robin=CASE["robin"], dirichlet=CASE["dirichlet"],
                            reactions=CASE["reactions"], init=init, graph=graph, sround=sround)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_reduced_storage_error(rd, oracle_mod):
    img, eps = _problem(seed=4)
    rng = np.random.default_rng(4)
    init = rng.uniform(0, 1, (1,) + img.shape)
    for storage, tol in (("bf16", 3e-2), ("fp16", 3e-3)):
        got, ref, _, _ = _run(rd, oracle_mod, img, eps, [1.0], 0.05, 100, 8, "column",
                              storage=storage, dirichlet={(0, 0): 1.0}, init=init, sround=True)
        err = rel_l2(got[0], ref[0], img != 0)
        print(f"{storage}: rel L2 {err:.3e}")
        assert err < tol


def test_constant_factor_equals_scaled_d(rd, oracle_mod):
    """e = 2 everywhere is D doubled (up to FP32 rounding order)."""
    img, _ = _problem(seed=12)
    rng = np.random.default_rng(12)
    init = rng.uniform(0, 1, (1,) + img.shape)
    got, _, _, _ = _run(rd, oracle_mod, img, np.full(img.shape, 2.0), [0.3], 0.1, 50, 8, "column",
                        dirichlet={(0, 0): 1.0}, init=init)
    _, s = make_gpu(rd, img, [0.6], dirichlet={(0, 0): 1.0}, kernel="column")
    c0 = oracle_mod.Problem(img, [0.6], dirichlet={(0, 0): 1.0}).apply_dirichlet(init)
    s.set_field(0, c0[0].astype(np.float32))
    s.step(0.1, 50)
    plain = fields(s, 1)
    assert rel_l2(got[0], plain[0], img != 0) < 1e-6


def test_smooth_diffusivity_from_sdf(rd, oracle_mod):
    """e from the signed distance on the GPU == the oracle's D(phi) rounded to FP32."""
    img, sdf = W.workload_geometry("spheres64")
    img = np.ascontiguousarray(img[:40, :37, :45])
    sdf = np.ascontiguousarray(sdf[:40, :37, :45]).astype(np.float32)
    pars = (0.05, 1.0, 0.5, 4.0)
    e_ref = oracle_mod.smooth_diffusivity(sdf.astype(np.float64), *pars).astype(np.float32)
    outs = []
    for mode in ("sdf", "values"):
        _, s = make_gpu(rd, img, [0.8], dirichlet={(0, 0): 1.0}, kernel="column",
                        features=rd.RD_WS_DIFFUSIVITY)
        if mode == "sdf":
            s.set_diffusivity_sdf(sdf, *pars)
        else:
            s.set_diffusivity(e_ref)
        s.step(0.1, 80)
        outs.append(fields(s, 1))
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-6
    prob = oracle_mod.Problem(img, [0.8], dirichlet={(0, 0): 1.0}, eps=e_ref.astype(np.float64))
    ref = prob.run(prob.initial(), 0.1, 80)
    assert rel_l2(outs[0][0], ref[0], img != 0) < TOL


def test_stability_bound_and_errors(rd):
    img = np.ones((8, 8, 8), np.uint8)
    _, s = make_gpu(rd, img, [1.0], features=rd.RD_WS_DIFFUSIVITY)
    s.step(0.15, 1)  # 2 / lambda_max = 1/6 with e = 1
    e = np.ones(img.shape, np.float32)
    e[3, 3, 3] = 2.0
    s.set_diffusivity(e)
    with pytest.raises(rd.RDError) as ex:
        s.step(0.15, 1)  # the bound is now 1/12
    assert ex.value.name == "RD_ERR_UNSTABLE_DT"
    s.step(0.08, 1)
    e[1, 2, 3] = -1.0
    with pytest.raises(rd.RDError) as ex:
        s.set_diffusivity(e)
    assert ex.value.name == "RD_ERR_ARG"
    s.step(0.15, 1)  # the factor was cleared
    e[1, 2, 3] = np.nan
    with pytest.raises(rd.RDError):
        s.set_diffusivity(e)
    s.clear_diffusivity()
    # a negative value on an inactive voxel is ignored
    img2 = img.copy()
    img2[1, 2, 3] = 0
    _, s2 = make_gpu(rd, img2, [1.0], features=rd.RD_WS_DIFFUSIVITY)
    e[1, 2, 3] = -1.0
    s2.set_diffusivity(e)
    # without the workspace feature
    _, s3 = make_gpu(rd, img, [1.0])
    with pytest.raises(rd.RDError) as ex:
        s3.set_diffusivity(np.ones(img.shape, np.float32))
    assert ex.value.name == "RD_ERR_WORKSPACE"
    # the steady state refuses a factor
    _, s4 = make_gpu(rd, img, [1.0], features=rd.RD_WS_DIFFUSIVITY | rd.RD_WS_SOLVER)
    s4.set_diffusivity(np.ones(img.shape, np.float32))
    with pytest.raises(rd.RDError) as ex:
        s4.steady_state(0, 1e-6, 1000)
    assert ex.value.name == "RD_ERR_STATE"


def test_mass_conserved_closed_box(rd):
    """No Dirichlet, Robin or reactions: FP64 mass of the FP32 field is conserved to
    rounding for any factor."""
    img, eps = _problem(seed=17, shape=(40, 33, 35))
    _, s = make_gpu(rd, img, [1.0], kernel="column", features=rd.RD_WS_DIFFUSIVITY)
    s.set_diffusivity(eps.astype(np.float32))
    rng = np.random.default_rng(17)
    s.set_field(0, rng.uniform(0, 1, img.shape).astype(np.float32))
    m0 = s.balance(0)["mass"]
    s.step(0.05, 400)
    m1 = s.balance(0)["mass"]
    assert abs(m1 - m0) < 1e-5 * m0


@pytest.mark.parametrize("B,kernel,with_factor", [(8, "column", True), (8, "column", False),
                                                  (4, "block", True), (8, "block", False)])
def test_sink_band_parity(rd, oracle_mod, B, kernel, with_factor):
    """Volumetric sink on the voxels next to the wall (phi < 1 voxel), with and without
    a diffusivity factor, against the oracle; balance terms on the same field."""
    img, eps = _problem(seed=41)
    phi = oracle_mod.signed_distance(img, 1.0)
    band = (img != 0) & (phi < 1.0)
    rng = np.random.default_rng(41)
    init = rng.uniform(0, 1, (2,) + img.shape)
    D = [1.0, 0.4]
    sink = {0: 0.2, 1: 0.05}
    dt = 0.04
    _, s = make_gpu(rd, img, D, 1.0, CASE["robin"], CASE["dirichlet"], CASE["reactions"], "fp32", B,
                    kernel=kernel, features=rd.RD_WS_DIFFUSIVITY)
    for sp, k in sink.items():
        s.set_sink(sp, k)
    if with_factor:
        s.set_diffusivity(eps.astype(np.float32))
    assert s.set_sink_band(phi, 1.0) == int(band.sum())
    prob = oracle_mod.Problem(img, D, robin=CASE["robin"], dirichlet=CASE["dirichlet"],
                              reactions=CASE["reactions"],
                              eps=eps.astype(np.float32).astype(np.float64) if with_factor else None,
                              sink=sink, sink_mask=band.astype(np.uint8))
    c0 = prob.apply_dirichlet(init)
    for sp in range(2):
        s.set_field(sp, c0[sp].astype(np.float32))
    s.step(dt, 60)
    got = fields(s, 2)
    ref = prob.run(c0, dt, 60)
    act = img != 0
    for sp in range(2):
        err = rel_l2(got[sp], ref[sp], act)
        print(f"sink B={B} {kernel} factor={with_factor} species {sp}: rel L2 {err:.3e}")
        assert err < TOL
    for sp in range(2):
        b = s.balance(sp)
        m, infl, up, re = prob.balance(got, sp)
        assert b["mass"] == pytest.approx(m, rel=1e-10, abs=1e-12)
        np.testing.assert_allclose(b["inflow"], infl, rtol=1e-9, atol=1e-12)
        assert b["uptake"] == pytest.approx(up, rel=1e-10, abs=1e-12)


def test_sink_band_kernels_agree_and_clear(rd, oracle_mod):
    img, _ = _problem(seed=43, shape=(26, 31, 35))
    phi = oracle_mod.signed_distance(img, 1.0)
    rng = np.random.default_rng(43)
    c0 = rng.uniform(0, 1, img.shape).astype(np.float32) * (img != 0)
    outs = []
    for kernel in ("column", "block"):
        _, s = make_gpu(rd, img, [1.0], kernel=kernel, features=rd.RD_WS_DIFFUSIVITY | rd.RD_WS_SOLVER)
        s.set_sink(0, 0.3)
        assert s.set_sink_band(phi, 1.6) > 0
        s.set_field(0, c0)
        s.step(0.05, 64)
        outs.append(fields(s, 1))
        with pytest.raises(rd.RDError) as ex:
            s.steady_state(0, 1e-6, 100)
        assert ex.value.name == "RD_ERR_STATE"
    assert np.array_equal(outs[0], outs[1])
    # an empty band gives back the constant-D step, bit for bit
    _, s = make_gpu(rd, img, [1.0], kernel="column", features=rd.RD_WS_DIFFUSIVITY)
    s.set_sink(0, 0.3)
    s.set_sink_band(phi, 1.6)
    assert s.set_sink_band(phi, 0.0) == 0
    s.set_field(0, c0)
    s.step(0.05, 64)
    _, p = make_gpu(rd, img, [1.0], kernel="column")
    p.set_field(0, c0)
    p.step(0.05, 64)
    assert np.array_equal(fields(s, 1), fields(p, 1))
    with pytest.raises(rd.RDError):
        s.set_sink(0, -1.0)


def test_autotune_keeps_factor_and_band(rd, oracle_mod):
    """The autotuner times the factor kernels, resets the fields only (the factor and the
    band marks stay), and its choice gives the bits of the default launch."""
    img, eps = _problem(seed=51, shape=(30, 34, 37))
    phi = oracle_mod.signed_distance(img, 1.0)
    rng = np.random.default_rng(51)
    c0 = (rng.uniform(0, 1, img.shape) * (img != 0)).astype(np.float32)
    outs = []
    for tune, band in ((False, 1.0), (True, 1.0), (False, 0.0)):
        _, s = make_gpu(rd, img, [1.0], dirichlet={(0, 0): 1.0}, kernel="column",
                        features=rd.RD_WS_DIFFUSIVITY)
        s.set_diffusivity(eps.astype(np.float32))
        s.set_sink(0, 0.2)
        s.set_sink_band(phi, band)
        if tune:
            s.autotune(0.04, 30)
            assert s.steps_taken() == 0
        s.set_field(0, c0)
        s.step(0.04, 100)
        outs.append(fields(s, 1))
    assert np.array_equal(outs[0], outs[1])
    assert not np.array_equal(outs[0], outs[2])  # the band's sink acts
