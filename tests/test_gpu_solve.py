"""Steady state and tortuosity on the GPU (conjugate gradients through the C ABI)
against the FP64 oracle's CG and against closed forms."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import fields, make_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _steady(rd, img, axis, storage="fp32", B=8, tol=1e-6, max_iters=20000):
    g, s = make_gpu(rd, img, [1.0], storage=storage, B=B, features=rd.RD_WS_SOLVER)
    res = s.steady_state(axis, tol, max_iters)
    return res, fields(s, 1)[0], s


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("B", [4, 8])
def test_straight_channels_tau_one(rd, axis, B):
    img = W.straight_channels(21, 14, 13, period=4, width=2)
    if axis == 1:
        img = np.ascontiguousarray(img.transpose(0, 2, 1))
    elif axis == 2:
        img = np.ascontiguousarray(img.transpose(2, 1, 0))
    res, u, _ = _steady(rd, img, axis, B=B)
    assert res["converged"], res
    # the FP64 ramp is the exact solution: tau = 1 to FP64 rounding
    assert res["tau"] == pytest.approx(1.0, rel=1e-12)


def test_non_percolating_tau_infinite(rd):
    img = W.slab_box(12, 6, 6)
    img[:, :, 5] = 0
    res, _, _ = _steady(rd, img, 0)
    assert math.isinf(res["tau"])


@pytest.mark.parametrize("n,seed", [(24, 1), (37, 2)])
def test_porous_tau_and_field_vs_oracle(rd, oracle_mod, n, seed):
    img, _ = W.boolean_spheres(n, 0.55, 2.0, 4.0, seed=seed)
    for axis in (0, 2):
        res, u, _ = _steady(rd, img, axis, tol=1e-6)
        uo, _, rel_o = oracle_mod.steady_state(img, axis, "cg", tol=1e-12)
        tau_o, qin, qout = oracle_mod.tortuosity_from_field(img, axis, uo)
        print(f"n={n} axis={axis}: GPU tau={res['tau']:.8f} (rel res {res['rel_residual']:.2e}, "
              f"{res['iters']} it), oracle tau={tau_o:.8f}")
        assert res["tau"] == pytest.approx(tau_o, rel=1e-4)
        # the steady field is unique only on clusters touching a Dirichlet plane
        assert rel_l2(u, uo, _anchored(img, axis)) < 1e-4


def _anchored(img, axis):
    from scipy import ndimage

    lab, _ = ndimage.label(img != 0)
    sl_lo = [slice(None)] * 3
    sl_hi = [slice(None)] * 3
    sl_lo[2 - axis] = 0
    sl_hi[2 - axis] = -1
    keep = np.union1d(np.unique(lab[tuple(sl_lo)]), np.unique(lab[tuple(sl_hi)]))
    keep = keep[keep > 0]
    return np.isin(lab, keep)


@pytest.mark.parametrize("B", [4, 8])
@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_refinement_reaches_1e8(rd, oracle_mod, storage, B):
    """Iterative refinement (FP64 solution and residual, CG corrections in the storage
    type) reaches the 1e-8 relative residual of the ceramic-foam configuration with
    every storage type; tau then agrees with the FP64 oracle's to the residual level."""
    img, _ = W.boolean_spheres(32, 0.6, 2.0, 4.0, seed=4)
    img = np.ascontiguousarray(img[:, :29, :])  # ragged
    uo, _, _ = oracle_mod.steady_state(img, 0, "cg", tol=1e-12)
    tau_o = oracle_mod.tortuosity_from_field(img, 0, uo)[0]
    res, u, _ = _steady(rd, img, 0, storage=storage, B=B, tol=1e-8, max_iters=20000)
    err = abs(res["tau"] - tau_o) / tau_o
    print(f"{storage} B={B}: rel residual {res['rel_residual']:.2e} after {res['iters']} it; "
          f"tau {res['tau']:.10f} vs {tau_o:.10f} (rel err {err:.2e})")
    assert res["converged"] and res["rel_residual"] <= 1e-8
    assert err < 1e-6
    # the field holds the FP64 solution rounded to the storage type
    spacing = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}[storage]
    assert rel_l2(u, uo, _anchored(img, 0)) < 2 * spacing


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_block_jacobi_preconditioner(rd, oracle_mod, storage):
    """CG with the block-Jacobi preconditioner (2 and 4 Jacobi steps per block) and plain
    CG reach the same steady state as the FP64 oracle, and the preconditioned runs need
    fewer iterations (the preconditioner changes the path, not the solution)."""
    img, _ = W.boolean_spheres(48, 0.6, 2.0, 5.0, seed=6)
    img = np.ascontiguousarray(img[:45, :, :43])  # ragged
    uo, _, _ = oracle_mod.steady_state(img, 0, "cg", tol=1e-12)
    tau_o = oracle_mod.tortuosity_from_field(img, 0, uo)[0]
    it = {}
    for k in (0, 2, 4):
        g, s = make_gpu(rd, img, [1.0], storage=storage, B=8, features=rd.RD_WS_SOLVER)
        s.set_cg_precond(k)
        res = s.steady_state(0, 1e-8, 20000)
        u = fields(s, 1)[0]
        err = abs(res["tau"] - tau_o) / tau_o
        print(f"{storage} jacobi steps {k}: rel residual {res['rel_residual']:.2e} after "
              f"{res['iters']} it; tau rel err {err:.2e}")
        assert res["converged"] and res["rel_residual"] <= 1e-8
        assert err < 1e-6
        spacing = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}[storage]
        assert rel_l2(u, uo, _anchored(img, 0)) < 2 * spacing
        it[k] = res["iters"]
    assert it[2] < it[0] and it[4] < it[0]


def test_precond_setting_checked(rd):
    img = W.slab_box(12, 6, 6)
    g, s = make_gpu(rd, img, [1.0], features=rd.RD_WS_SOLVER)
    for bad in (-1, 17):
        with pytest.raises(rd.RDError, match="ARG"):
            s.set_cg_precond(bad)


@pytest.mark.parametrize("steps", [0, 2])
def test_batch_precond_setting_matches_single(rd, steps):
    """A batch run with a given preconditioner setting gives each geometry the bits of its
    single-geometry run with the same setting (plain CG and 2 Jacobi steps)."""
    imgs = [W.boolean_spheres(n, 0.55, 2.0, 4.0, seed=40 + n)[0] for n in (19, 26, 13)]
    bt = rd.Batch([rd.Geometry(im, None, 1.0, 8) for im in imgs]).bind()
    bt.set_cg_precond(steps)
    tau, rel, it = bt.tortuosity(0, 1e-8, 20000)
    for i, im in enumerate(imgs):
        g, s = make_gpu(rd, im, [1.0], features=rd.RD_WS_SOLVER)
        s.set_cg_precond(steps)
        res = s.steady_state(0, 1e-8, 20000)
        assert res["converged"] and rel[i] <= 1e-8
        assert tau[i] == res["tau"] and it[i] == res["iters"]
    with pytest.raises(rd.RDError, match="ARG"):
        bt.set_cg_precond(17)


def test_batch_matches_single_and_oracle(rd, oracle_mod):
    imgs = []
    for i, n in enumerate([17, 24, 9, 31, 20]):
        img, _ = W.boolean_spheres(n, 0.5 + 0.05 * i, 2.0, 4.0, seed=10 + i)
        imgs.append(img)
    imgs.append(W.straight_channels(16, 12, 12))
    geoms = [rd.Geometry(im, None, 1.0, 8) for im in imgs]
    bt = rd.Batch(geoms).bind()
    tau, rel, it = bt.tortuosity(0, 1e-6, 20000)
    for i, im in enumerate(imgs):
        res, _, _ = _steady(rd, im, 0, tol=1e-6)
        uo, _, _ = oracle_mod.steady_state(im, 0, "cg", tol=1e-12)
        tau_o = oracle_mod.tortuosity_from_field(im, 0, uo)[0]
        print(f"geometry {i}: batch tau {tau[i]:.7f} single {res['tau']:.7f} oracle {tau_o:.7f}")
        if math.isinf(tau_o):
            assert math.isinf(tau[i])
            continue
        assert tau[i] == pytest.approx(tau_o, rel=1e-4)
        # the batch runs the single-geometry arithmetic per geometry: same bits
        assert tau[i] == res["tau"] and it[i] == res["iters"]
    assert tau[-1] == pytest.approx(1.0, rel=1e-5)
    assert np.all(np.asarray(rel) <= 1e-6)  # every geometry reaches the tolerance


@pytest.mark.parametrize("B", [4, 8])
def test_batch_degenerate_members(rd, oracle_mod, B):
    """A batch holding an empty geometry, one that does not percolate, a single voxel
    and a normal packing: the degenerate members give tau = inf without disturbing the
    others, whose tau equals the oracle's."""
    empty = np.zeros((9, 10, 11), np.uint8)
    blocked = W.slab_box(12, 6, 6)
    blocked[:, :, 5] = 0
    one = np.zeros((5, 5, 5), np.uint8)
    one[2, 2, 2] = 1
    pack, _ = W.boolean_spheres(21, 0.55, 2.0, 4.0, seed=33)
    imgs = [empty, pack, blocked, one, pack]
    geoms = [rd.Geometry(im, None, 1.0, B) for im in imgs]
    bt = rd.Batch(geoms).bind()
    tau, rel, it = bt.tortuosity(0, 1e-8, 20000)
    uo, _, _ = oracle_mod.steady_state(pack, 0, "cg", tol=1e-12)
    tau_o = oracle_mod.tortuosity_from_field(pack, 0, uo)[0]
    print(f"B={B}: tau {list(tau)}, rel {list(rel)}, iters {list(it)}; oracle {tau_o:.10f}")
    assert math.isinf(tau[0]) and math.isinf(tau[2]) and math.isinf(tau[3])
    assert tau[1] == pytest.approx(tau_o, rel=1e-7) and tau[4] == tau[1]
    assert rel[1] <= 1e-8 and rel[4] <= 1e-8


def _expected_guess(img, axis):
    """The cluster rule of the initial guess, from scipy's 6-connected labelling (an
    independent implementation): inlet plane 1, outlet plane 0; inside, the ramp
    1 - c/(n-1) on clusters touching both planes, 1 on clusters touching only the
    inlet, 0 elsewhere (the ramp in FP64, rounded to FP32 as on the GPU)."""
    from scipy import ndimage

    act = img != 0
    lab, _ = ndimage.label(act, structure=ndimage.generate_binary_structure(3, 1))
    ax = 2 - axis  # array axes are (z, y, x)
    n = img.shape[ax]
    c = np.indices(img.shape)[ax]
    lo = np.take(lab, 0, axis=ax)
    hi = np.take(lab, n - 1, axis=ax)
    tin = np.isin(lab, lo[lo > 0])
    tout = np.isin(lab, hi[hi > 0])
    ramp = (1.0 - c / (n - 1)).astype(np.float32)  # the exact ramp, rounded once
    g = np.where(tin & tout, ramp, np.where(tin, np.float32(1), np.float32(0))).astype(np.float32)
    g[c == 0] = 1.0
    g[c == n - 1] = 0.0
    g[~act] = 0.0
    return g, bool(np.any(tin & tout))


@pytest.mark.parametrize("B", [4, 8])
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_initial_guess_cluster_rule(rd, B, storage, axis):
    """The GPU labelling gives the cluster rule exactly (max_iters = 0 leaves the guess
    in the field): a random packing with floating and inlet-only clusters, plus a
    floating block of voxels and an inlet-only bar added by hand."""
    from gpu_common import round_to_storage

    img, _ = W.boolean_spheres(30, 0.35, 2.0, 4.0, seed=7)
    img = np.ascontiguousarray(img[:27, :25, :])  # ragged: (nz, ny, nx) = (27, 25, 30)
    img[10:13, 10:13, 10:13] = 1
    img[9:14, 9:14, 9] = 0; img[9:14, 9:14, 13] = 0  # isolate a 3^3 cube
    img[9:14, 9, 9:14] = 0; img[9:14, 13, 9:14] = 0
    img[9, 9:14, 9:14] = 0; img[13, 9:14, 9:14] = 0
    img[0:3, 0:3, 0:3] = 1  # a corner cube on every inlet plane, cut off from the rest
    img[0:4, 0:4, 3] = 0; img[0:4, 3, 0:4] = 0; img[3, 0:4, 0:4] = 0
    want, perc = _expected_guess(img, axis)
    c = np.indices(img.shape)[2 - axis]
    assert np.any((want == 1.0) & (c > 0)) and np.any((want == 0.0) & (img != 0) & (c < c.max()))
    g, s = make_gpu(rd, img, [1.0], storage=storage, B=B, features=rd.RD_WS_SOLVER)
    res = s.steady_state(axis, 1e-6, 0)
    got = fields(s, 1)[0]
    np.testing.assert_array_equal(got, round_to_storage(want, storage))
    assert math.isinf(res["tau"]) != perc


def test_batch_autotune_pick(rd, oracle_mod):
    """The batch autotuner times both block edges and leaves batches that still give the
    oracle's tau."""
    imgs = [W.boolean_spheres(n, 0.5, 2.0, 4.0, seed=40 + n)[0] for n in (19, 26, 33)]
    batches = [rd.Batch([rd.Geometry(im, None, 1.0, B) for im in imgs]).bind() for B in (8, 4)]
    best, ms = rd.batch_autotune_pick(batches, 0, 30)
    print(f"batch autotune: 8^3 {ms[0]:.4f} ms/it, 4^3 {ms[1]:.4f} ms/it, best {best}")
    assert best in (0, 1) and np.all(ms > 0)
    for bt in batches:
        tau, rel, _ = bt.tortuosity(0, 1e-8, 20000)
        for i, im in enumerate(imgs):
            uo, _, _ = oracle_mod.steady_state(im, 0, "cg", tol=1e-12)
            tau_o = oracle_mod.tortuosity_from_field(im, 0, uo)[0]
            assert tau[i] == pytest.approx(tau_o, rel=1e-7)


def test_batch_launch_settings(rd, oracle_mod):
    """The batch's CG segment replayed as a captured graph gives the bits of direct
    launches; 50 iterations per check stops at other points but reaches the oracle's tau."""
    imgs = [W.boolean_spheres(n, 0.5, 2.0, 4.0, seed=70 + n)[0] for n in (18, 27, 35)]
    geoms = [rd.Geometry(im, None, 1.0, 8) for im in imgs]
    res = {}
    for every, graph in ((25, True), (25, False), (50, True)):
        bt = rd.Batch(geoms).bind().set_launch(every, graph)
        assert bt.get_launch() == {"iters_per_check": every, "use_graph": int(graph)}
        res[(every, graph)] = bt.tortuosity(0, 1e-8, 20000)
    np.testing.assert_array_equal(res[(25, True)][0], res[(25, False)][0])
    np.testing.assert_array_equal(res[(25, True)][2], res[(25, False)][2])
    assert np.all(res[(50, True)][2] % 50 == 0)
    for i, im in enumerate(imgs):
        uo, _, _ = oracle_mod.steady_state(im, 0, "cg", tol=1e-12)
        tau_o = oracle_mod.tortuosity_from_field(im, 0, uo)[0]
        for key, (tau, rel, it) in res.items():
            assert tau[i] == pytest.approx(tau_o, rel=1e-7), key
            assert rel[i] <= 1e-8
