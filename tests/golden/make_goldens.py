"""Write the stored expected values of the full-size parity tests.

Every number written here comes from the FP64 oracle (``oracle/``) run on the seeded
volumes of ``workloads``; nothing is taken from the HIP library.  The oracle's sums are
formed per z-plane and added in plane order, so the values do not depend on the thread
count.  Each output file records the SHA-256 of the volume it was computed on; the tests
refuse to compare against a file whose volume they cannot regenerate bit for bit.

    python tests/golden/make_goldens.py foam_crop256   # steady state, three axes
    python tests/golden/make_goldens.py batch64        # tortuosity of the 64 packings
    python tests/golden/make_goldens.py decay256       # adjoint and central differences
    python tests/golden/make_goldens.py decay256_fd_half  # central differences at h / 2
    python tests/golden/make_goldens.py soil512        # 512^3 soil, 1000 and 10000 steps

Cost on 8 host cores: foam_crop256 a few minutes, batch64 about 20 minutes, decay256
about 15 minutes, soil512 about 80 minutes.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def sha(img):
    return hashlib.sha256(np.ascontiguousarray(img, dtype=np.uint8).tobytes()).hexdigest()


def _write_json(name, obj):
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


# ---------------------------------------------------------------------------
# C3: the ceramic-foam recipe, a 256^3 corner crop of the 1024^3 volume
# ---------------------------------------------------------------------------

FOAM_CROP = 256


def foam_crop(n=FOAM_CROP):
    """The corner (n^3) of the 1024^3 ceramic-foam volume (solid matrix active)."""
    img, _ = W.workload_geometry("foam1024")
    return np.ascontiguousarray(img[:n, :n, :n])


def make_foam_crop256():
    img = foam_crop()
    out = {"_about": "FP64 oracle CG (rel. residual 1e-12) on the 256^3 corner crop of the "
                     "1024^3 ceramic-foam volume (active = solid matrix), unit drop along each "
                     "axis; tau = psi D dT A / (Q L) (eq. tortuosity)",
           "shape": list(img.shape), "sha256": sha(img),
           "active_fraction": float(img.mean()), "axes": {}}
    for axis in (0, 1, 2):
        t = time.time()
        u, it, rel = oracle.steady_state(img, axis, "cg", tol=1e-12)
        tau, qin, qout = oracle.tortuosity_from_field(img, axis, u)
        out["axes"][str(axis)] = {"tau": tau, "q_in": qin, "q_out": qout, "iters": it,
                                  "rel_residual": rel}
        print(f"foam crop axis {axis}: tau {tau:.12f} ({it} it, rel {rel:.2e}, "
              f"{time.time() - t:.1f} s)", flush=True)
    _write_json("foam_crop256_tau.json", out)


# ---------------------------------------------------------------------------
# C4: the 64 sphere packings of the batched workload
# ---------------------------------------------------------------------------

def make_batch64():
    geoms = W.batch_geometries()
    out = {"_about": "FP64 oracle CG (rel. residual 1e-12) tortuosity along x of the 64 "
                     "boolean sphere packings of the batched workload (seed stream (4, i))",
           "members": []}
    for i, (img, info) in enumerate(geoms):
        t = time.time()
        u, it, rel = oracle.steady_state(img, 0, "cg", tol=1e-12)
        tau, qin, qout = oracle.tortuosity_from_field(img, 0, u)
        out["members"].append({"i": i, "n": info["n"], "sha256": sha(img),
                               "active_fraction": float(img.mean()),
                               "tau": None if math.isinf(tau) else tau,
                               "q_in": qin, "q_out": qout, "iters": it, "rel_residual": rel})
        print(f"packing {i}: n {info['n']} tau {tau:.10f} ({it} it, {time.time() - t:.1f} s)",
              flush=True)
    _write_json("batch64_tau.json", out)


# ---------------------------------------------------------------------------
# C5: adjoint of diffusion-decay on the 256^3 packing
# ---------------------------------------------------------------------------

def decay_target(img, w, steps=None):
    """Target field c* of the adjoint workload: the FP64 oracle's state after the
    workload's steps with D = 1 and decay rate 0.01, rounded to FP32."""
    prob = oracle.Problem(img, [1.0], dirichlet=w.dirichlet, reactions=[(0, -1, 0.01)])
    return prob.run(prob.initial(), w.dt, steps or w.steps)[0].astype(np.float32)


def decay_loss(img, w, D, k, target):
    """L = 1/2 sum over free voxels (c^N - c*)^2 of the FP64 oracle's forward run."""
    prob = oracle.Problem(img, [D], dirichlet=w.dirichlet, reactions=[(0, -1, k)])
    cN = prob.run(prob.initial(), w.dt, w.steps)[0]
    free = prob.free_mask(0)
    d = (cN - target.astype(np.float64))[free]
    return 0.5 * float(np.sum(d * d))


def make_decay256():
    w = W.workload("decay256")
    img, _ = W.workload_geometry("decay256")
    t = time.time()
    target = decay_target(img, w)
    print(f"target: {time.time() - t:.1f} s", flush=True)
    D, k, h = 0.8, 0.02, 1e-3
    prob = oracle.Problem(img, [D], dirichlet=w.dirichlet)
    t = time.time()
    L, gD, gk, _ = oracle.adjoint_decay(img, D, k, w.dt, w.steps, prob.initial()[0],
                                        target.astype(np.float64), stride=50)
    print(f"adjoint: L {L:.12e} dL/dD {gD:.12e} dL/dk {gk:.12e} ({time.time() - t:.1f} s)",
          flush=True)
    fd = {}
    for name, (dp, dm) in {"D": ((D + h, k), (D - h, k)), "k": ((D, k + h), (D, k - h))}.items():
        t = time.time()
        lp = decay_loss(img, w, *dp, target)
        lm = decay_loss(img, w, *dm, target)
        fd[name] = {"L_plus": lp, "L_minus": lm, "central": (lp - lm) / (2 * h)}
        print(f"central difference d/d{name}: {fd[name]['central']:.12e} ({time.time() - t:.1f} s)",
              flush=True)
    _write_json("decay256_adjoint.json", {
        "_about": "FP64 oracle on the 256^3 diffusion-decay packing (p = 0.5, seed 5): target "
                  "from D = 1, k = 0.01 after 2000 steps (stored as FP32), loss and gradients "
                  "at D = 0.8, k = 0.02 from the oracle adjoint (checkpoint stride 50) and from "
                  "central differences of the oracle loss with h = 1e-3",
        "shape": list(img.shape), "sha256": sha(img), "D": D, "k": k, "dt": w.dt,
        "steps": w.steps, "h": h, "loss": L, "dL_dD": gD, "dL_dk": gk, "fd": fd,
        "target_sum": float(np.sum(target.astype(np.float64)))})


def make_decay256_fd_half():
    """Central differences with h / 2 added to decay256_adjoint.json: with the ones at h
    they give the Richardson value (4 D(h/2) - D(h)) / 3, whose truncation error is
    O(h^4) (the one at h alone is O(h^2): about (h/k)^2 relative in k = 0.02)."""
    path = os.path.join(HERE, "decay256_adjoint.json")
    ref = json.load(open(path))
    w = W.workload("decay256")
    img, _ = W.workload_geometry("decay256")
    assert sha(img) == ref["sha256"]
    target = decay_target(img, w)
    assert float(np.sum(target.astype(np.float64))) == ref["target_sum"]
    D, k, h = ref["D"], ref["k"], ref["h"] / 2
    for name, (dp, dm) in {"D": ((D + h, k), (D - h, k)), "k": ((D, k + h), (D, k - h))}.items():
        t = time.time()
        lp = decay_loss(img, w, *dp, target)
        lm = decay_loss(img, w, *dm, target)
        half = (lp - lm) / (2 * h)
        ref["fd"][name].update({"L_plus_half": lp, "L_minus_half": lm, "central_half": half,
                                "richardson": (4 * half - ref["fd"][name]["central"]) / 3})
        print(f"central difference d/d{name} with h/2: {half:.12e}, Richardson "
              f"{ref['fd'][name]['richardson']:.12e} ({time.time() - t:.1f} s)", flush=True)
    _write_json("decay256_adjoint.json", ref)


# ---------------------------------------------------------------------------
# C2: 512^3 soil volume, two species, 1000 and 10000 steps
# ---------------------------------------------------------------------------

SOIL_SAMPLE_SEED = 20230422
SOIL_NEAR = 4096   # samples among the active voxels with x < 192 (the front's reach)
SOIL_FAR = 1024    # samples among all active voxels


def soil_samples(img):
    """Flat indices of the sampled voxels (seeded; near the inlet and over the volume)."""
    rng = np.random.default_rng(SOIL_SAMPLE_SEED)
    act = np.flatnonzero(img.ravel() != 0)
    x = act % img.shape[2]
    near = act[x < 192]
    a = np.sort(rng.choice(near, SOIL_NEAR, replace=False))
    b = np.sort(rng.choice(act, SOIL_FAR, replace=False))
    return np.concatenate([a, b]).astype(np.int64)


def make_soil512():
    w = W.workload("soil512")
    img, _ = W.workload_geometry("soil512")
    prob = oracle.Problem(img, w.species_D, robin=w.robin, dirichlet=w.dirichlet,
                          reactions=w.reactions)
    idx = soil_samples(img)
    c = prob.initial()
    rec = {}
    done = 0
    for n in (1000, w.steps):
        t = time.time()
        c = prob.run(c, w.dt, n - done)
        done = n
        print(f"soil512: {n} steps ({time.time() - t:.1f} s)", flush=True)
        flat = c.reshape(c.shape[0], -1)
        rec[f"samples_{n}"] = np.stack([flat[s][idx] for s in range(c.shape[0])])
        # c is (species, nz, ny, nx): mass per x-plane (along the inflow) and per z-plane
        rec[f"xprofile_{n}"] = c.sum(axis=(1, 2))
        rec[f"zprofile_{n}"] = c.sum(axis=(2, 3))
        for s in range(c.shape[0]):
            m, inflow, up, re = prob.balance(c, s)
            rec[f"balance_{n}_{s}"] = np.array([m, *inflow, up, re])
    np.savez_compressed(os.path.join(HERE, "soil512_oracle.npz"), index=idx,
                        sha256=np.array(sha(img)), **rec)
    print("wrote soil512_oracle.npz", flush=True)


if __name__ == "__main__":
    jobs = {"foam_crop256": make_foam_crop256, "batch64": make_batch64,
            "decay256": make_decay256, "decay256_fd_half": make_decay256_fd_half,
            "soil512": make_soil512}
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
