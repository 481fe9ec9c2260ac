"""Parity at the workloads' own sizes and step counts.

Live FP64 oracle runs where the oracle finishes in about a minute:
* the soil recipe (Gaussian random field, correlation length 12, porosity 0.3, two
  species, A -> B, Robin uptake of B, inlet c_A = 1) on a 128^3 volume for the full
  10 000 steps, every active voxel compared;
* the ceramic-foam recipe (solid matrix of a boolean model of pore balls r ~ U(10, 30))
  on a 144^3 volume (5832 blocks of 8^3, so the single-geometry solver takes its
  two-level segment sums), steady field and tortuosity.

Stored oracle values (``tests/golden/make_goldens.py``, which calls only the oracle)
where the full size is beyond a test's time:
* 512^3 soil volume after 1000 and 10 000 steps: 5120 sampled voxels per species, the
  mass per x-plane and per z-plane and the balance terms;
* the 256^3 corner crop of the 1024^3 foam: tortuosity along x, y and z with FP32
  storage, along x with FP16 storage (eq. tortuosity);
* the 64 sphere packings of the batched workload: tortuosity along x;
* the 256^3 diffusion-decay packing: loss and gradients from the oracle adjoint and from
  central differences of the oracle loss (h = 1e-3 and 1e-3 / 2, and their Richardson value), after 2000 steps with checkpoints
  every 100.
Each stored file names the SHA-256 of its volume; the regenerated volume must match.
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import rel_l2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sha(img):
    return hashlib.sha256(np.ascontiguousarray(img, dtype=np.uint8).tobytes()).hexdigest()


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"stored oracle values {name} not generated (tests/golden/make_goldens.py)")
    return path


def _json(name):
    with open(_golden(name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _soil_sim(rd, img, w, stochastic=True):
    g = rd.Geometry(img, None, w.dx, 8)
    s = rd.Sim(g, "fp32")
    if stochastic:  # the benchmark's setting
        s.set_rounding(1, seed=2304)
    for d in w.species_D:
        s.add_species(d)
    for (a, b, k) in w.reactions:
        s.add_reaction(a, b, k)
    for sp, k in w.robin.items():
        s.set_robin(sp, k)
    for (sp, f), v in w.dirichlet.items():
        s.set_dirichlet(sp, f, v)
    s.bind()
    s.autotune(w.dt, 100)  # the launch the benchmark times
    return g, s


def _fields(s, n):
    return np.stack([s.get_field(i).cpu().numpy() for i in range(n)]).astype(np.float64)


# ---------------------------------------------------------------------------
# soil recipe, two species, 10 000 steps
# ---------------------------------------------------------------------------

def test_soil128_full_step_count_vs_oracle(rd, oracle_mod):
    """FP32 storage with stochastic rounding (the benchmark's setting) after the full
    10 000 steps; round to nearest beside it.  As the field settles, the increments of a
    step fall below half an FP32 ulp and round to nearest drops them, so that run stalls
    near (ulp / 2) / (dt * decay rate) from the FP64 solution; the dithered rounding keeps
    them on average."""
    w = W.workload("soil512")
    img = W.gaussian_random_field_volume(128, 12.0, 0.3, seed=w.seed)
    prob = oracle_mod.Problem(img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                              reactions=w.reactions)
    ref = prob.run(prob.initial(), w.dt, w.steps)
    act = img != 0
    errs = {}
    for stochastic in (True, False):
        g, s = _soil_sim(rd, img, w, stochastic)
        s.step(w.dt, w.steps)
        got = _fields(s, 2)
        assert np.all(got[:, ~act] == 0)
        errs[stochastic] = [rel_l2(got[sp], ref[sp], act) for sp in range(2)]
        print(f"soil 128^3, {w.steps} steps, {'stochastic' if stochastic else 'nearest'} "
              f"rounding: rel L2 A {errs[stochastic][0]:.3e} B {errs[stochastic][1]:.3e}")
    # measured: stochastic 3.9e-7 / 2.7e-7, nearest 8.9e-6 / 1.5e-5
    assert max(errs[True]) <= 2e-6
    assert max(errs[True]) * 10 < max(errs[False])


def test_soil512_vs_stored_oracle(rd):
    w = W.workload("soil512")
    img, _ = W.workload_geometry("soil512")
    ref = np.load(_golden("soil512_oracle.npz"))
    assert _sha(img) == str(ref["sha256"]), "the 512^3 soil volume differs from the stored one"
    idx = ref["index"]
    g, s = _soil_sim(rd, img, w)
    for n in (1000, w.steps):
        s.step(w.dt, n - s.steps_taken())
        assert s.steps_taken() == n
        got = _fields(s, 2)
        flat = got.reshape(2, -1)
        want = ref[f"samples_{n}"]
        prof = {"x": got.sum(axis=(1, 2)), "z": got.sum(axis=(2, 3))}  # got: (2, nz, ny, nx)
        for sp in range(2):
            a, b = flat[sp][idx], want[sp]
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            perr = {}
            for ax in "xz":
                o = ref[f"{ax}profile_{n}"][sp]
                perr[ax] = np.linalg.norm(prof[ax][sp] - o) / np.linalg.norm(o)
            bal = s.balance(sp)
            ob = ref[f"balance_{n}_{sp}"]
            print(f"soil 512^3, {n} steps, species {sp}: sampled rel L2 {err:.3e}, mass per "
                  f"x-plane rel L2 {perr['x']:.3e}, per z-plane {perr['z']:.3e}, mass "
                  f"{bal['mass']:.6f} (oracle {ob[0]:.6f})")
            assert err <= 1e-5 and max(perr.values()) <= 1e-5
            assert bal["mass"] == pytest.approx(ob[0], rel=1e-5)
            assert bal["uptake"] == pytest.approx(ob[7], rel=1e-5, abs=1e-9)
            assert np.allclose(bal["inflow"], ob[1:7], rtol=1e-5, atol=1e-9)


# ---------------------------------------------------------------------------
# ceramic-foam recipe: steady state and tortuosity
# ---------------------------------------------------------------------------

def _steady(rd, img, axis, storage, tol=1e-8):
    g = rd.Geometry(img, None, 1.0, 8)
    s = rd.Sim(g, storage)
    s.add_species(1.0)
    s.bind(features=rd.RD_WS_SOLVER)
    nb = g.stats()["n_blocks"]
    return s.steady_state(axis, tol, 100000), s, nb


def test_foam144_steady_field_vs_oracle(rd, oracle_mod):
    from test_gpu_solve import _anchored

    img, _ = W.boolean_spheres(144, 0.15, 10.0, 30.0, seed=3, active="solid")
    res, s, nb = _steady(rd, img, 0, "fp32")
    assert nb > 4096  # the two-level segment sums
    u = s.get_field(0).cpu().numpy().astype(np.float64)
    uo, it, rel = oracle_mod.steady_state(img, 0, "cg", tol=1e-12)
    tau_o = oracle_mod.tortuosity_from_field(img, 0, uo)[0]
    err = rel_l2(u, uo, _anchored(img, 0))
    print(f"foam 144^3 ({nb} blocks): tau {res['tau']:.10f} vs oracle {tau_o:.10f}; field rel L2 "
          f"{err:.2e}; residual {res['rel_residual']:.2e} after {res['iters']} it")
    assert res["converged"] and res["rel_residual"] <= 1e-8
    # a relative residual of 1e-8 leaves tau about 1e-7 from the converged value (measured
    # 1.9e-7)
    assert res["tau"] == pytest.approx(tau_o, rel=1e-6)
    assert err <= 1e-6


@pytest.fixture(scope="module")
def foam_crop():
    from make_goldens import foam_crop as crop

    img = crop()
    ref = _json("foam_crop256_tau.json")
    assert _sha(img) == ref["sha256"], "the foam crop differs from the stored one"
    return img, ref


# BF16 vectors reach 1e-8 on the foam with the block-Jacobi preconditioner (plain CG stalled
# near 2e-5 on the 1024^3 volume: the 8-bit mantissa of the directions)
@pytest.mark.parametrize("storage,axis", [("fp32", 0), ("fp32", 1), ("fp32", 2), ("fp16", 0), ("bf16", 0)])
def test_foam_crop256_tau_vs_stored_oracle(rd, foam_crop, storage, axis):
    img, ref = foam_crop
    res, s, nb = _steady(rd, img, axis, storage)
    tau_o = ref["axes"][str(axis)]["tau"]
    err = abs(res["tau"] - tau_o) / tau_o
    print(f"foam crop 256^3 ({nb} blocks) {storage} axis {axis}: tau {res['tau']:.10f} vs oracle "
          f"{tau_o:.10f} (rel {err:.2e}); residual {res['rel_residual']:.2e}, {res['iters']} it")
    assert nb > 4096
    assert res["converged"] and res["rel_residual"] <= 1e-8
    assert err <= 1e-6


# ---------------------------------------------------------------------------
# batched form: the 64 packings
# ---------------------------------------------------------------------------

def test_batch64_tau_vs_stored_oracle(rd):
    """All 64 packings in one batch against the oracle's tau (CG to 1e-12).  The batched
    benchmark solves to a relative residual of 1e-6 with 25 or 50 iterations per check
    (graph and direct launches give the same bits, test_gpu_solve); at 1e-6 the measured
    tau error reaches 1e-4 on the largest packings, so each setting is checked there against
    2e-4, and once more solved to 1e-8, where tau must agree to 2e-6 (measured 4.5e-7)."""
    ref = _json("batch64_tau.json")["members"]
    geoms = W.batch_geometries()
    assert len(geoms) == len(ref) == 64
    for (img, info), r in zip(geoms, ref):
        assert _sha(img) == r["sha256"], f"packing {r['i']} differs from the stored one"
    hs = [rd.Geometry(img, None, 1.0, 8) for img, _ in geoms]
    bt = rd.Batch(hs).bind()
    for every, use_graph, tol, bar in ((50, False, 1e-6, 2e-4), (25, True, 1e-6, 2e-4),
                                       (25, True, 1e-8, 2e-6)):
        bt.set_launch(every, use_graph)
        tau, rel, it = bt.tortuosity(0, tol, 100000)
        errs = []
        for i, r in enumerate(ref):
            if r["tau"] is None:
                assert math.isinf(tau[i])
                continue
            errs.append(abs(tau[i] - r["tau"]) / r["tau"])
        print(f"batch of 64, {every} iterations per check, tolerance {tol:g}: max tau rel err "
              f"{max(errs):.2e}, median {np.median(errs):.2e}; largest final residual "
              f"{np.max(rel):.2e}; iterations {int(np.min(it))}..{int(np.max(it))}")
        assert np.all(rel <= tol)
        assert max(errs) <= bar


# ---------------------------------------------------------------------------
# adjoint: the 256^3 diffusion-decay packing
# ---------------------------------------------------------------------------

def test_decay256_adjoint_vs_stored_oracle(rd):
    from make_goldens import decay_target

    ref = _json("decay256_adjoint.json")
    w = W.workload("decay256")
    img, _ = W.workload_geometry("decay256")
    assert _sha(img) == ref["sha256"], "the 256^3 packing differs from the stored one"
    target = decay_target(img, w)
    assert float(np.sum(target.astype(np.float64))) == ref["target_sum"]
    every = 100
    g = rd.Geometry(img, None, w.dx, 8)
    s = rd.Sim(g, "fp32")
    s.add_species(ref["D"])
    s.add_reaction(0, -1, ref["k"])
    for (sp, f), v in w.dirichlet.items():
        s.set_dirichlet(sp, f, v)
    s.bind(features=rd.RD_WS_ADJOINT, checkpoint_slots=-(-w.steps // every) + every - 1)
    L, gD, gk = s.adjoint(target, w.steps, w.dt, every)
    eD = abs(gD - ref["dL_dD"]) / abs(ref["dL_dD"])
    ek = abs(gk - ref["dL_dk"]) / abs(ref["dL_dk"])
    fD = abs(gD - ref["fd"]["D"]["central"]) / abs(ref["fd"]["D"]["central"])
    fk = abs(gk - ref["fd"]["k"]["central"]) / abs(ref["fd"]["k"]["central"])
    print(f"decay 256^3: loss {L:.10e} vs {ref['loss']:.10e}; dL/dD {gD:.10e} vs adjoint "
          f"{ref['dL_dD']:.10e} (rel {eD:.2e}) vs central differences {ref['fd']['D']['central']:.10e} "
          f"(rel {fD:.2e}); dL/dk {gk:.10e} vs {ref['dL_dk']:.10e} (rel {ek:.2e}) vs "
          f"{ref['fd']['k']['central']:.10e} (rel {fk:.2e})")
    # measured: loss 5.2e-7, dL/dD 3.5e-7, dL/dk 1.8e-7
    assert L == pytest.approx(ref["loss"], rel=2e-6)
    assert eD <= 2e-6 and ek <= 2e-6
    # central differences with h = 1e-3 carry an O(h^2) truncation error: 1e-6 relative in
    # D = 0.8, but about (h / k)^2 = 2.5e-3 in k = 0.02 (the oracle's own adjoint and its
    # differences differ by 5.8e-4 there); the Richardson value of h and h / 2 is O(h^4)
    assert fD <= 1e-5 and fk <= 2e-3
    for name, g in (("D", gD), ("k", gk)):
        rich = ref["fd"][name]["richardson"]
        err = abs(g - rich) / abs(rich)
        print(f"dL/d{name} vs Richardson central differences {rich:.10e}: rel {err:.2e}")
        assert err <= 2e-6  # measured 3.5e-7 (D), 3.1e-7 (k)
