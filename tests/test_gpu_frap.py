"""Simulated FRAP on the GPU (region mass of the bleached box while the field
recovers, section "Calculation of effective diffusion coefficient and tortuosity")
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from gpu_common import fields, make_gpu, round_to_storage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _geom(seed=3, shape=(19, 23, 29)):
    img, _ = W.boolean_spheres(max(shape), 0.6, 2.0, 4.0, seed=seed)
    return np.ascontiguousarray(img[:shape[0], :shape[1], :shape[2]])


@pytest.mark.parametrize("B", [4, 8])
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_region_mass(rd, oracle_mod, B, storage):
    img = _geom()
    nz, ny, nx = img.shape
    rng = np.random.default_rng(B)
    _, s = make_gpu(rd, img, [1.0], B=B, storage=storage, dx=0.5)
    c = round_to_storage(rng.uniform(0, 1, img.shape), storage)
    s.set_field(0, c.astype(np.float32))
    got = fields(s, 1)[0]
    regions = [(0, nx, 0, ny, 0, nz), (3, 17, 5, 9, 7, 16), (7, 9, 0, 23, 8, 9),
               (28, 29, 22, 23, 18, 19), (8, 16, 8, 16, 8, 16)]
    for reg in regions:
        want = oracle_mod.region_mass(img, got, reg, 0.5)
        assert s.region_mass(0, reg) == pytest.approx(want, rel=1e-12, abs=1e-14), reg
    for bad in [(0, 0, 0, ny, 0, nz), (0, nx + 1, 0, ny, 0, nz), (-1, 3, 0, 1, 0, 1)]:
        with pytest.raises(rd.RDError):
            s.region_mass(0, bad)


def _bleached(img, reg):
    x0, x1, y0, y1, z0, z1 = reg
    c = (img != 0).astype(np.float64)
    c[z0:z1, y0:y1, x0:x1] = 0.0
    return c


@pytest.mark.parametrize("B", [4, 8])
def test_frap_curve(rd, oracle_mod, B):
    img = _geom(seed=5, shape=(30, 30, 30))
    reg = (10, 20, 10, 20, 10, 20)
    c0 = _bleached(img, reg)
    _, s = make_gpu(rd, img, [1.0], B=B, kernel="column" if B == 8 else "block")
    s.set_field(0, c0.astype(np.float32))
    got = s.frap_curve(0, reg, 0.1, 10, 30)
    prob = oracle_mod.Problem(img, [1.0])
    ref = oracle_mod.frap_curve(prob, c0[None], reg, 0.1, 10, 30)
    assert got[0] == ref[0] == 0.0
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_frap_tortuosity_end_to_end(rd, oracle_mod):
    """Porous and free-space curves on the GPU, fitted by the library == the same
    pipeline in the oracle (curves and SciPy fit)."""
    n = 32
    img = _geom(seed=11, shape=(n, n, n))
    bulk = np.ones_like(img)
    reg = (12, 20, 12, 20, 12, 20)
    dt, sps, ns = 0.1, 10, 40

    def norm(curve, im):
        c0 = _bleached(im, reg)
        x0, x1, y0, y1, z0, z1 = reg
        cinf = c0.sum() / (im != 0).sum()
        return curve / (cinf * (im[z0:z1, y0:y1, x0:x1] != 0).sum())

    curves = {}
    for name, im, sps_i, ns_i in (("por", img, sps, ns), ("bulk", bulk, 2, 5 * ns)):
        _, s = make_gpu(rd, im, [1.0], kernel="column")
        s.set_field(0, _bleached(im, reg).astype(np.float32))
        g = norm(s.frap_curve(0, reg, dt, sps_i, ns_i), im)
        prob = oracle_mod.Problem(im, [1.0])
        r = norm(oracle_mod.frap_curve(prob, _bleached(im, reg)[None], reg, dt, sps_i, ns_i), im)
        np.testing.assert_allclose(g, r, rtol=1e-5, atol=1e-6)
        curves[name] = (g, r)
    t = np.arange(ns + 1) * sps * dt
    d_gpu, rms = rd.frap_fit(t, curves["por"][0], 2 * dt, curves["bulk"][0], 1.0)
    d_ora = oracle_mod.frap_fit(t, curves["por"][1], 2 * dt, curves["bulk"][1], 1.0)
    print(f"FRAP D_eff gpu {d_gpu:.6f} oracle {d_ora:.6f} tau {1 / d_gpu:.4f} rms {rms:.2e}")
    assert d_gpu == pytest.approx(d_ora, rel=1e-4)
    assert 0.2 < d_gpu < 1.0


def test_frap_curve_with_factor_and_sink(rd, oracle_mod):
    """FRAP recovery with the smooth D(phi) factor and a sink band (the paper's two
    application examples' ingredients) against the oracle."""
    img = _geom(seed=17, shape=(28, 30, 26))
    reg = (9, 17, 10, 20, 8, 18)
    c0 = _bleached(img, reg)
    phi = oracle_mod.signed_distance(img, 1.0)
    eps = oracle_mod.smooth_diffusivity(phi.astype(np.float64), 0.1, 0.9, -6.0, 4.0).astype(np.float32)
    band = (img != 0) & (phi < 1.0)
    _, s = make_gpu(rd, img, [1.0], kernel="column", features=rd.RD_WS_DIFFUSIVITY)
    s.set_diffusivity(eps)
    s.set_sink(0, 0.01)
    assert s.set_sink_band(phi, 1.0) == int(band.sum())
    s.set_field(0, c0.astype(np.float32))
    got = s.frap_curve(0, reg, 0.1, 10, 25)
    prob = oracle_mod.Problem(img, [1.0], eps=eps.astype(np.float64), sink={0: 0.01},
                              sink_mask=band.astype(np.uint8))
    ref = oracle_mod.frap_curve(prob, c0[None], reg, 0.1, 10, 25)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_edge_cases(rd, oracle_mod):
    """The whole box's region mass is the balance's mass; an empty geometry accepts a
    factor, a band and FRAP calls; a one-voxel region."""
    img = _geom(seed=23, shape=(21, 18, 27))
    nz, ny, nx = img.shape
    _, s = make_gpu(rd, img, [1.0], dirichlet={(0, 0): 0.7}, features=rd.RD_WS_DIFFUSIVITY)
    rng = np.random.default_rng(23)
    s.set_field(0, rng.uniform(0, 1, img.shape).astype(np.float32))
    s.step(0.1, 5)
    got = fields(s, 1)[0]
    free = (img != 0).copy()
    free[:, :, 0] = False  # Dirichlet plane: not part of the balance's mass
    whole = s.region_mass(0, (0, nx, 0, ny, 0, nz))
    assert whole == pytest.approx(oracle_mod.region_mass(img, got, (0, nx, 0, ny, 0, nz)), rel=1e-12)
    assert s.region_mass(0, (1, nx, 0, ny, 0, nz)) == pytest.approx(s.balance(0)["mass"], rel=1e-12)
    p = tuple(np.argwhere(img != 0)[7])
    one = (p[2], p[2] + 1, p[1], p[1] + 1, p[0], p[0] + 1)
    assert s.region_mass(0, one) == pytest.approx(got[p], rel=1e-7)
    # empty geometry
    empty = np.zeros((9, 10, 11), np.uint8)
    _, e = make_gpu(rd, empty, [1.0], features=rd.RD_WS_DIFFUSIVITY)
    e.set_diffusivity(np.ones(empty.shape, np.float32))
    assert e.set_sink_band(np.ones(empty.shape, np.float32), 2.0) == 0
    e.step(0.1, 3)
    assert e.region_mass(0, (0, 11, 0, 10, 0, 9)) == 0.0
    assert np.all(e.frap_curve(0, (2, 5, 2, 5, 2, 5), 0.1, 2, 3) == 0.0)
