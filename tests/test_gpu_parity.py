"""GPU (HIP, through the C ABI) vs the FP64 oracle, element by element.

Tolerance: relative L2 over active voxels <= 1e-5 for FP32 storage after the
workload's steps (FP32 rounding of ~1e-7 per step, damped by diffusion).
"""
import math

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


def _run_both(rd, oracle_mod, img, D, dt, n, B=8, dx=1.0, robin=None, dirichlet=None,
              reactions=None, init=None, storage="fp32", graph=True, kernel="block"):
    g, s = make_gpu(rd, img, D, dx, robin, dirichlet, reactions, storage, B, graph=graph,
                    kernel=kernel)
    prob = oracle_mod.Problem(img, D, dx=dx, robin=robin, dirichlet=dirichlet, reactions=reactions)
    c0 = prob.initial()
    if init is not None:
        c0 = prob.apply_dirichlet(round_to_storage(init, storage))
        for sp in range(len(D)):
            s.set_field(sp, c0[sp].astype(np.float32))
    s.step(dt, n)
    got = fields(s, len(D))
    ref = prob.run(c0, dt, n)
    return got, ref, prob, s


def test_slab_closed_form_and_oracle(rd, oracle_mod):
    N = 37  # ragged: not a multiple of 4 or 8
    img = W.slab_box(N, ny=5, nz=3)
    for B in (4, 8):
        got, ref, _, _ = _run_both(rd, oracle_mod, img, [1.0], 0.1, 400, B=B, dirichlet={(0, 0): 1.0})
        act = img != 0
        assert rel_l2(got[0], ref[0], act) < TOL
        i = np.arange(N)
        u = np.ones(N)
        for m in range(N - 1):
            th = (2 * m + 1) * math.pi / (2 * N - 1)
            a = -np.sin(th * i[1:]).sum() / ((2 * N - 1) / 4.0)
            u += a * (1 - 4 * 0.1 * math.sin(th / 2) ** 2) ** 400 * np.sin(th * i)
        np.testing.assert_allclose(got[0, 1, 2], u, atol=2e-6)


def test_spheres64_full_config(rd, oracle_mod):
    """64^3 disjoint-sphere packing, D = 1, dt = 0.1, 1000 steps, c = 1 on x = 0."""
    w = W.workload("spheres64")
    img, sdf = W.workload_geometry("spheres64")
    g, s = make_gpu(rd, img, w.species_D, w.dx, dirichlet=w.dirichlet, B=8, sdf=sdf)
    s.step(w.dt, w.steps)
    got8 = fields(s, 1)
    prob = oracle_mod.Problem(img, w.species_D, dirichlet=w.dirichlet)
    ref = prob.run(prob.initial(), w.dt, w.steps)
    act = img != 0
    err = rel_l2(got8[0], ref[0], act)
    print(f"spheres64 rel L2 = {err:.3e}")
    assert err < TOL
    assert np.all(got8[0][~act] == 0)
    # every kernel variant gives the same bits: B = 4, one workgroup per block,
    # plain or XCD-aware mapping, graph replay or direct launches, grid sizes
    variants = [dict(B=4, graph=False), dict(B=4, xcd=False), dict(kernel="persistent"),
                dict(kernel="persistent", xcd=False), dict(xcd=False, graph=False),
                dict(kernel="persistent", wg_per_cu=1), dict(kernel="persistent", wg_per_cu=3, xcd=False),
                dict(kernel="column"), dict(kernel="column", xcd=False, graph=False),
                dict(kernel="column_xch"), dict(kernel="column_xch", xcd=False, graph=False)]
    for v in variants:
        _, sv = make_gpu(rd, img, w.species_D, w.dx, dirichlet=w.dirichlet, **v)
        sv.step(w.dt, w.steps)
        np.testing.assert_array_equal(fields(sv, 1), got8, err_msg=str(v))


def test_soil_reduced_two_species(rd, oracle_mod):
    """Soil recipe at 96^3: A, B with D = (1, 0.4), A -> B at 0.01, Robin on B."""
    w = W.workload("soil512", small=True)
    img, _ = W.workload_geometry("soil512", small=True)
    got, ref, prob, s = _run_both(rd, oracle_mod, img, w.species_D, w.dt, 1500, B=8,
                                  robin=w.robin, dirichlet=w.dirichlet, reactions=w.reactions)
    act = img != 0
    for sp in range(2):
        err = rel_l2(got[sp], ref[sp], act)
        print(f"soil96 species {sp} rel L2 = {err:.3e}")
        assert err < TOL
    # FP64 balance terms of the GPU field agree with the oracle's on the same field
    for sp in range(2):
        b = s.balance(sp)
        m, infl, up, re = prob.balance(got, sp)
        assert b["mass"] == pytest.approx(m, rel=1e-10)
        np.testing.assert_allclose(b["inflow"], infl, rtol=1e-9, atol=1e-9)
        assert b["uptake"] == pytest.approx(up, rel=1e-10, abs=1e-12)
        assert b["react"] == pytest.approx(re, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("seed", range(12))
def test_random_tiny_geometries(rd, oracle_mod, seed):
    """Edge cases: sizes not a multiple of B, isolated voxels, thin walls, random
    stable parameters and random initial fields."""
    rng = np.random.default_rng(100 + seed)
    img = W.random_tiny_geometry(seed)
    S = int(rng.integers(1, 4))
    D = list(rng.uniform(0.1, 1.0, S))
    dx = float(rng.uniform(0.5, 2.0))
    robin = {int(rng.integers(0, S)): float(rng.uniform(0, 0.2))}
    reactions = [(0, -1, float(rng.uniform(0, 0.05)))]
    if S > 1:
        reactions.append((0, 1, float(rng.uniform(0, 0.05))))
    dirichlet = {(int(rng.integers(0, S)), int(rng.integers(0, 6))): float(rng.uniform(0, 1))}
    lam = 12 * max(D) / dx ** 2 + sum(r[2] for r in reactions) + 6 * max(robin.values()) / dx
    dt = 1.9 / lam
    init = rng.uniform(0, 1, (S,) + img.shape)
    for B, kernel in ((4, "block"), (8, "block"), (8, "column"), (8, "column_xch")):
        got, ref, prob, s = _run_both(rd, oracle_mod, img, D, dt, 60, B=B, dx=dx, robin=robin,
                                      dirichlet=dirichlet, reactions=reactions, init=init,
                                      kernel=kernel)
        assert np.abs(got - ref).max() < 2e-5, (seed, B, kernel)
        _check_balance(s, prob, got, S)


def _check_balance(s, prob, got, S):
    """FP64 balance terms of the GPU field equal the oracle's on the same field."""
    for sp in range(S):
        b = s.balance(sp)
        m, infl, up, re = prob.balance(got, sp)
        assert b["mass"] == pytest.approx(m, rel=1e-10, abs=1e-12)
        np.testing.assert_allclose(b["inflow"], infl, rtol=1e-9, atol=1e-12)
        assert b["uptake"] == pytest.approx(up, rel=1e-10, abs=1e-12)
        assert b["react"] == pytest.approx(re, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_balance_dirichlet_every_face_ragged(rd, oracle_mod, storage):
    """Dirichlet data on all six faces of a box whose edges are 1 mod 8: the inflow of a
    + face plane alone in its block comes from the neighbouring block."""
    img, _ = W.boolean_spheres(49, 0.5, 2.0, 4.0, seed=21)
    img = np.ascontiguousarray(img[:33, :41, :])  # (nz, ny, nx) = (33, 41, 49)
    rng = np.random.default_rng(21)
    dirichlet = {(0, f): float(rng.uniform(0.2, 1.0)) for f in range(6)}
    dirichlet[(1, 1)] = 0.7
    dirichlet[(1, 5)] = 0.3
    reactions = [(0, 1, 0.02), (1, -1, 0.01)]
    robin = {1: 0.05}
    init = rng.uniform(0, 1, (2,) + img.shape)
    for B in (4, 8):
        got, ref, prob, s = _run_both(rd, oracle_mod, img, [1.0, 0.5], 0.1, 40, B=B,
                                      robin=robin, dirichlet=dirichlet, reactions=reactions,
                                      init=init, storage=storage, kernel="column" if B == 8 else "block")
        assert np.all(np.array(s.balance(0)["inflow"]) != 0.0)
        _check_balance(s, prob, got, 2)
        # plane fluxes, including planes on block boundaries (i0 = 7, 15: the +axis
        # neighbour lies in the next block) and the last plane of each axis
        for axis, n in ((0, img.shape[2]), (1, img.shape[1]), (2, img.shape[0])):
            for i0 in (0, 3, 7, 8, 15, n // 2, n - 2):
                for sp in range(2):
                    want = prob.plane_flux(got[sp], [1.0, 0.5][sp], axis, i0)
                    assert s.plane_flux(sp, axis, i0) == pytest.approx(want, rel=1e-10, abs=1e-13), \
                        (B, storage, axis, i0, sp)
        with pytest.raises(rd.RDError):
            s.plane_flux(0, 0, img.shape[2] - 1)


def test_empty_and_single_voxel(rd, oracle_mod):
    img = np.zeros((9, 10, 11), np.uint8)
    g, s = make_gpu(rd, img, [1.0])
    s.step(0.1, 5)
    assert np.all(fields(s, 1) == 0)
    assert s.balance(0)["mass"] == 0.0
    img[4, 5, 6] = 1
    got, ref, _, _ = _run_both(rd, oracle_mod, img, [1.0], 0.1, 50, robin={0: 0.1},
                               init=np.ones((1,) + img.shape))
    assert got[0, 4, 5, 6] == pytest.approx(ref[0, 4, 5, 6], rel=1e-5)
    assert ref[0, 4, 5, 6] == pytest.approx((1 - 0.1 * 0.1 * 6) ** 50, rel=1e-12)


def test_mass_conservation_fp32(rd, oracle_mod):
    img, _ = W.boolean_spheres(48, 0.5, 3.0, 6.0, seed=11)
    rng = np.random.default_rng(11)
    init = rng.uniform(0, 1, (1,) + img.shape)
    g, s = make_gpu(rd, img, [1.0])
    s.set_field(0, (init[0] * (img != 0)).astype(np.float32))
    m0 = s.balance(0)["mass"]
    s.step(0.15, 2000)
    m1 = s.balance(0)["mass"]
    drift = abs(m1 - m0) / m0 / 2000
    print(f"FP32 normalised mass drift per step = {drift:.3e} (paper, FP32 on A100: 7.91e-10)")
    assert drift < 1e-8


def test_deterministic_and_resume(rd, oracle_mod):
    w = W.workload("soil512", small=True)
    img, _ = W.workload_geometry("soil512", small=True)
    runs = []
    for _ in range(2):
        _, s = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                        reactions=w.reactions)
        s.step(w.dt, 300)
        runs.append(fields(s, 2))
    np.testing.assert_array_equal(runs[0], runs[1])
    # interrupt after 100 steps, save with get_field, restore with set_field
    _, s = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                    reactions=w.reactions)
    s.step(w.dt, 100)
    saved = [s.get_field(i).clone() for i in range(2)]
    _, s2 = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                     reactions=w.reactions)
    for i in range(2):
        s2.set_field(i, saved[i])
    s2.step(w.dt, 200)
    np.testing.assert_array_equal(fields(s2, 2), runs[0])


def test_error_paths(rd):
    img = np.ones((8, 8, 8), np.uint8)
    _, s = make_gpu(rd, img, [1.0])
    with pytest.raises(rd.RDError) as e:
        s.step(0.2, 1)  # 2/lambda_max = 1/6
    assert e.value.name == "RD_ERR_UNSTABLE_DT"
    with pytest.raises(rd.RDError):
        s.get_field(3)
    bad = np.zeros((8, 8, 8), np.float32)
    bad[2, 3, 4] = np.nan
    s.set_field(0, bad)
    with pytest.raises(rd.RDError) as e:
        s.balance(0)
    assert e.value.name == "RD_ERR_NONFINITE"


@pytest.mark.parametrize("storage", ["bf16", "fp16"])
def test_reduced_storage_error_reported(rd, oracle_mod, storage):
    """BF16 / FP16 storage with FP32 arithmetic on the 64^3 packing (1000 steps).

    Parity unpinned: the error against the FP64 oracle is measured and reported.
    Round-to-nearest storage loses increments below half a storage spacing, so the
    front stalls; stochastic rounding is unbiased and must stay within a few
    storage spacings (bounds: BF16 spacing 2^-8, FP16 2^-11 in [0.5, 1))."""
    w = W.workload("spheres64")
    img, sdf = W.workload_geometry("spheres64")
    prob = oracle_mod.Problem(img, w.species_D, dirichlet=w.dirichlet)
    ref = prob.run(prob.initial(), w.dt, w.steps)
    act = img != 0
    errs = {}
    for sr in (0, 1):
        g, s = make_gpu(rd, img, w.species_D, dirichlet=w.dirichlet, storage=storage)
        s.set_rounding(sr, seed=1234)
        s.step(w.dt, w.steps)
        errs[sr] = rel_l2(fields(s, 1)[0], ref[0], act)
    print(f"spheres64 {storage}: rel L2 vs FP64 nearest = {errs[0]:.3e}, stochastic = {errs[1]:.3e}")
    bound = {"bf16": 2 ** -8, "fp16": 2 ** -11}[storage] * 4
    assert errs[1] < bound
    assert errs[1] < errs[0]


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_stochastic_rounding_variants_agree(rd, storage):
    """Stochastic rounding draws its bits from (slot, species, step, seed), so graph
    replay, direct launches and every kernel variant round identically (FP32: the
    dithered increment; BF16 / FP16: the store)."""
    img, _ = W.boolean_spheres(40, 0.5, 3.0, 6.0, seed=3)
    out = []
    for v in [dict(), dict(graph=False), dict(kernel="persistent"), dict(B=4),
              dict(kernel="persistent", wg_per_cu=2), dict(kernel="column"),
              dict(kernel="column_xch")]:
        g, s = make_gpu(rd, img, [1.0, 0.5], dirichlet={(0, 0): 1.0}, reactions=[(0, 1, 0.02)],
                        storage=storage, **v)
        s.set_rounding(1, seed=99)
        s.step(0.1, 77)
        out.append(fields(s, 2))
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("S", [1, 3, 4])
def test_species_counts_and_storage_kernels_agree(rd, oracle_mod, storage, S):
    """Each (storage, species count) instantiation of the persistent B = 8 kernel
    equals the one-block-per-workgroup kernel and the B = 4 kernel bit for bit, and
    FP32 matches the oracle."""
    img, _ = W.boolean_spheres((21, 26, 35), 0.6, 2.0, 4.0, seed=S)
    rng = np.random.default_rng(S)
    D = list(rng.uniform(0.2, 1.0, S))
    reactions = [(i, i + 1, 0.03) for i in range(S - 1)] + [(0, -1, 0.01)]
    robin = {S - 1: 0.04}
    dirichlet = {(0, 0): 1.0, (S - 1, 5): 0.5}
    init = rng.uniform(0, 1, (S,) + img.shape).astype(np.float32)
    out = []
    for v in [dict(), dict(kernel="persistent"), dict(B=4), dict(kernel="column"),
              dict(kernel="column_xch")]:
        g, s = make_gpu(rd, img, D, robin=robin, dirichlet=dirichlet, reactions=reactions,
                        storage=storage, **v)
        for sp in range(S):
            s.set_field(sp, init[sp])
        s.step(0.1, 40)
        out.append(fields(s, S))
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])
    if storage == "fp32":
        prob = oracle_mod.Problem(img, D, robin=robin, dirichlet=dirichlet, reactions=reactions)
        ref = prob.run(prob.apply_dirichlet(init.astype(np.float64)), 0.1, 40)
        assert np.abs(out[0] - ref).max() < 1e-5


def test_autotune_resets_and_matches(rd):
    """The autotuner keeps a launch setting that gives the same bits as the default and
    resets the fields; picking between 4^3 and 8^3 indexings returns a valid choice."""
    w = W.workload("soil512", small=True)
    img, _ = W.workload_geometry("soil512", small=True)
    _, ref = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                      reactions=w.reactions)
    ref.step(w.dt, 150)
    want = fields(ref, 2)
    sims = []
    for B in (8, 4):
        _, s = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                        reactions=w.reactions, B=B)
        sims.append(s)
    best, ms = rd.autotune_pick(sims, w.dt, 40)
    print(f"autotune: B=8 {ms[0]:.4f} ms/step, B=4 {ms[1]:.4f} ms/step, best index {best}, "
          f"launch {sims[best].get_launch()}")
    assert best in (0, 1) and np.all(ms > 0)
    for s in sims:
        assert s.steps_taken() == 0
        assert s.balance(1)["mass"] == 0.0  # reset: B is zero everywhere
        s.step(w.dt, 150)
        np.testing.assert_array_equal(fields(s, 2), want)


def test_autotune_cache(rd, tmp_path):
    """A tuned launch is stored under a key of GPU, storage, species and geometry: the
    same geometry bound again gets it without trials, another geometry does not, and
    the cached launch still gives the default launch's bits."""
    w = W.workload("soil512", small=True)
    img, _ = W.workload_geometry("soil512", small=True)
    cache = tmp_path / "tune.txt"

    def sim(image):
        return make_gpu(rd, image, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                        reactions=w.reactions)[1]

    s1 = sim(img)
    ms1 = s1.autotune(w.dt, 30, cache_path=cache)
    assert not s1.last_tune_from_cache and ms1 > 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("rdtune1 ")
    s2 = sim(img)
    ms2 = s2.autotune(w.dt, 30, cache_path=cache)
    assert s2.last_tune_from_cache and ms2 == pytest.approx(ms1, rel=1e-5)
    assert s2.get_launch() == s1.get_launch()
    other = img.copy()
    other[0, 0, 0] = 1 - other[0, 0, 0]
    s3 = sim(other)
    s3.autotune(w.dt, 30, cache_path=cache)
    assert not s3.last_tune_from_cache and len(cache.read_text().splitlines()) == 2
    _, ref = make_gpu(rd, img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                      reactions=w.reactions)
    ref.step(w.dt, 100)
    s2.step(w.dt, 100)
    np.testing.assert_array_equal(fields(s2, 2), fields(ref, 2))
