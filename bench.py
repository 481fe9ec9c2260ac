#!/usr/bin/env python3
"""Benchmark: explicit FTCS reaction-diffusion on a sparse block grid, one MI355X.

Headline workload: a 512^3 soil-like volume (seeded Gaussian random field,
correlation length 12 voxels, thresholded to porosity 0.3), 8^3 blocks, species A
and B with D = (1.0, 0.4), A -> B at rate 0.01, Robin wall uptake of B with
k = 0.05, c_A = 1 on the x = 0 face, dt = 0.1, FP32 storage.  One "step" is one
FTCS time step of both species over the whole geometry (the workload is 10 000
steps; that is the default --steps).

The JSON line carries: active-voxel updates/s (value); the step kernel's achieved
HBM bandwidth on algorithmic bytes (2 x 4 B x species per active voxel) over the
average launch time measured with HIP events on the launch stream, against the
8 TB/s peak (roofline); the same workload with BF16 / FP16 storage (stochastic
rounding) and its error against the FP32-storage run; a batched form (per-geometry
tortuosity of several sphere packings in one set of launches); and the FP64 CPU
oracle timed on a bounded sample of the headline workload (cpu_baseline).

Modes: --profile (only the timed loop of one storage type, FP32 unless --profile-storage,
for rocprofv3), --copy-calibration (a
plain 1 GiB device copy, whose FETCH_SIZE / WRITE_SIZE counters calibrate the
traffic figures).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "step_traffic.json")
STEP_SOURCES = ["paper_2304_11165_amd/csrc/k_step.hip", "paper_2304_11165_amd/csrc/rd_device.h",
                "paper_2304_11165_amd/csrc/rd_internal.h"]
METRIC = "active-voxel updates/s + achieved HBM GB/s (plain FP32 vs batched/BF16 form)"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--size", type=int, default=512, help="edge of the volume (default 512)")
    p.add_argument("--forms", default="bf16,fp16", help="reduced-storage forms to time")
    p.add_argument("--form-steps", type=int, default=2000)
    p.add_argument("--batch", type=int, default=64, help="geometries in the batched form (0: skip)")
    p.add_argument("--batch-max-edge", type=int, default=256)
    p.add_argument("--batch-steps", type=int, default=200,
                   help="time steps of the batched stepping form (0: skip)")
    p.add_argument("--fused-steps", type=int, default=16,
                   help="steps per cooperative launch in the fused form (0: skip the form)")
    p.add_argument("--steady-axes", type=int, default=1,
                   help="ceramic-foam steady state: tortuosity along the first K axes (0: skip)")
    p.add_argument("--steady-size", type=int, default=1024, help="edge of the foam volume")
    p.add_argument("--steady-forms", default="fp32,fp16,bf16", help="storage types of the steady form")
    p.add_argument("--steady-crop-forms", default="fp32,fp16,bf16",
                   help="storage types of the check on the foam's 256^3 crop against the stored oracle tau")
    p.add_argument("--steady-tol", type=float, default=1e-8)
    p.add_argument("--steady-max-iters", type=int, default=200000)
    p.add_argument("--cg-precond", type=int, default=6,
                   help="Jacobi steps of the steady-state CG's block preconditioner (0: plain CG)")
    p.add_argument("--adjoint", type=int, default=1,
                   help="1: time the checkpointed adjoint on the 256^3 diffusion-decay packing")
    p.add_argument("--diffusivity-steps", type=int, default=2000,
                   help="FP32 steps of the inhomogeneous-diffusion form (smooth D(phi) on the "
                        "same volume, phi built on the GPU; 0: skip)")
    p.add_argument("--frap-size", type=int, default=0,
                   help="edge of the volume of the simulated-FRAP form (0: skip)")
    p.add_argument("--cpu-steps", type=int, default=0,
                   help="oracle steps in the CPU sample (0: as many as fit in --cpu-seconds)")
    p.add_argument("--cpu-seconds", type=float, default=5.0,
                   help="target length of each of the three all-thread CPU samples when "
                        "--cpu-steps is 0")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--graph-steps", type=int, default=32)
    p.add_argument("--no-graph", action="store_true", help="direct launches (for profilers)")
    p.add_argument("--profile", action="store_true", help="only the timed FP32 loop")
    p.add_argument("--profile-storage", default="fp32", choices=["fp32", "bf16", "fp16"],
                   help="storage type timed by --profile")
    p.add_argument("--copy-calibration", action="store_true")
    p.add_argument("--profile-form", default="",
                   choices=["", "steady", "batch", "batch_steps", "fused", "adjoint"],
                   help="run only this form (for rocprofv3) and print its record")
    p.add_argument("--kernel", default="auto", choices=["auto", "block", "column", "column_xch",
                                                        "persistent", "column_lanes"],
                   help="B = 8 step kernel (auto: autotuned)")
    p.add_argument("--layout", default="auto", choices=["auto", "blocks", "compact"],
                   help="field layout (auto: the faster of the two, each autotuned)")
    p.add_argument("--xcd", default="auto", choices=["auto", "0", "1"],
                   help="XCD-aware block order (auto: autotuned)")
    p.add_argument("--traffic", default=TRAFFIC_FILE,
                   help="JSON records of measured HBM bytes per step launch (rocprofv3 FETCH_SIZE + "
                        "WRITE_SIZE, copy-calibrated), per kernel and block order; used only if the "
                        "kernel sources still match")
    return p.parse_args()


def source_hash():
    """Hash of the sources the step kernel is built from (a traffic record is valid only
    for the code it was measured on)."""
    import hashlib

    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(path, kernel, workload, xcd_map):
    """HBM bytes per launch from the traffic records (one per kernel and block order), or
    None if none was measured on this code, kernel, block order and workload."""
    if not path or not os.path.exists(path):
        return None
    recs = json.load(open(path)).get("records", [])
    for rec in recs:
        if rec.get("source_hash") == source_hash() and rec.get("kernel") == kernel and \
                rec.get("workload") == workload and rec.get("xcd_map") == int(xcd_map):
            return rec.get("hbm_bytes_per_launch")
    log(f"no traffic record in {path} for these sources, kernel {kernel}, block order {int(xcd_map)} "
        f"and workload: traffic = null")
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration():
    """A plain device copy of 1 GiB (read 1 GiB + write 1 GiB per launch), 20 launches."""
    import torch

    n = (1 << 30) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / 20
    print(json.dumps({"copy_bytes_per_launch": 2 * (1 << 30), "copy_GBps": 2 * (1 << 30) / t / 1e9}))


def build_sim(rd, geom, w, storage, graph_steps, use_graph=True):
    s = rd.Sim(geom, storage)
    for d in w.species_D:
        s.add_species(d)
    for (a, b, k) in w.reactions:
        s.add_reaction(a, b, k)
    for sp, k in w.robin.items():
        s.set_robin(sp, k)
    for (sp, f), v in w.dirichlet.items():
        s.set_dirichlet(sp, f, v)
    s.set_launch(graph_steps, use_graph, True)
    # stochastic rounding for every storage type (FP32: a dither of the increment), so
    # increments below half a storage spacing are not lost as the field settles
    s.set_rounding(1, seed=2304)
    return s


def time_steps(torch, sim, stream, dt, warmup, steps):
    """Warm-up, then exactly `steps` steps timed with HIP events on the launch stream.
    The steps are issued in chunks with an event between chunks: chunks of one captured
    graph (the launch's steps per graph) when there are at least ten of them, else
    single steps launched directly.  Returns (seconds, wall seconds, timing record with
    the mean and standard error of the per-chunk time per step)."""
    import math

    sim.step(dt, warmup)
    torch.cuda.synchronize()
    launch = sim.get_launch()
    gs = launch["graph_steps"] + (launch["graph_steps"] & 1)
    chunk = gs if (launch["use_graph"] and steps >= 10 * gs) else 1
    sizes = [chunk] * (steps // chunk) + ([steps % chunk] if steps % chunk else [])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(sizes) + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i, n in enumerate(sizes):
        sim.step(dt, n)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    secs = ev[0].elapsed_time(ev[-1]) / 1e3
    per = [ev[i].elapsed_time(ev[i + 1]) / n for i, n in enumerate(sizes) if n == chunk]
    mean = sum(per) / len(per)
    se = math.sqrt(sum((x - mean) ** 2 for x in per) / (len(per) - 1) / len(per)) if len(per) > 1 else 0.0
    timing = {"chunks": len(per), "steps_per_chunk": chunk,
              "launches": "captured graphs" if chunk > 1 else "direct launches",
              "ms_per_step_mean": mean, "ms_per_step_stderr": se}
    return secs, wall, timing


def step_kernel_name(B, launch, S):
    """HIP kernel that runs the FP32 step under a launch setting (B = 4 has one)."""
    if B == 4:
        return f"k_step4w<float,{S}>"
    kern = (launch or {}).get("kernel", "block")
    cmp = "true" if (launch or {}).get("layout") == "compact" else "false"
    d = "true"  # FP32 with stochastic rounding: the dithered instantiation
    name = {"block": "k_step8<float,{S},{D}>", "column": "k_step8z<float,{S},false,{C},{D}>",
            "column_xch": "k_step8z<float,{S},true,{C},{D}>", "persistent": "k_step8p<float,{S},{D}>",
            "column_lanes": "k_step8l<float,{S},{D}>"}[kern]
    return name.format(S=S, C=cmp, D=d)


def cg_words(prec):
    """Vector words per active voxel and CG iteration: the matvec with the p update fused
    (reads p and z, or r without the preconditioner; writes p) and the x, r update with
    A p recomputed (reads x, p, r; writes x, r, and z with the preconditioner)."""
    return 9 if prec > 0 else 8


def batched_form(torch, rd, W, count, max_edge, stream, prec=6):
    """Per-geometry tortuosity along x of `count` boolean sphere packings (edge
    U{64..max_edge}, porosity U(0.3, 0.7)), all in one set of CG launches."""
    t0 = time.perf_counter()
    geoms_np = W.batch_geometries(count, seed=4, nmin=64, nmax=max_edge)
    # 8^3 blocks only: the 4^3 CG kernels (one thread per slot, A p stored) took 7.6 ms
    # per iteration of this batch against 2.3 ms for the 8^3 column kernels
    edges = (8,)
    cands = {B: [rd.Geometry(img, None, 1.0, B) for img, _ in geoms_np] for B in edges}
    n_active = sum(g.stats()["n_active"] for g in cands[8])
    log(f"batch of {count}: generated and indexed in {time.perf_counter() - t0:.1f}s, {n_active} active voxels")
    with torch.cuda.stream(stream):
        # launch setting (iterations per graph segment, graph replay) by the batch
        # autotuner (50 CG iterations per trial)
        batches = [rd.Batch(cands[B]).bind(stream=stream) for B in edges]
        for bt in batches:
            bt.set_cg_precond(prec)
        best, trial_ms = rd.batch_autotune_pick(batches, 0, 50)
        bt, geoms, block_edge = batches[best], cands[edges[best]], edges[best]
        launch = bt.get_launch()
        del batches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tau, rel, it = bt.tortuosity(0, 1e-6, 20000)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
    voxel_iters = float(sum(g.stats()["n_active"] * int(i) for g, i in zip(geoms, it)))
    log(f"batched: block edge {block_edge}, launch {launch} (trial ms per iteration: "
        f"{', '.join(f'{B}^3 {m:.3f}' for B, m in zip(edges, trial_ms))})")
    return {
        "geometries": count,
        "block_edge": block_edge,
        "launch": launch,
        "cg_precond_jacobi_steps": prec,
        "trial_ms_per_iteration": {f"{B}^3": float(m) for B, m in zip(edges, trial_ms)},
        "edges": [int(info["n"]) for _, info in geoms_np],
        "seconds": secs,
        "active_voxel_cg_iterations_per_s": voxel_iters / secs,
        "alg_GBps": voxel_iters * cg_words(prec) * 4 / secs / 1e9,
        "tau": [float(x) for x in tau],
        "rel_residual_max": float(max(rel)),
        "iterations": [int(x) for x in it],
        "note": "wall time of the tortuosity call: cluster labelling, initial guess and CG",
    }


def batched_step_form(torch, rd, W, count, max_edge, steps, stream):
    """Time stepping of `count` sphere packings (the batched form's volumes) with the soil
    recipe (two species, A -> B, Robin uptake of B, c_A = 1 on each packing's x = 0 face,
    FP32 with stochastic rounding): one concatenated geometry stepped in shared launches
    against each packing stepped on its own with the same launch setting."""
    w = W.workload("soil512")
    t0 = time.perf_counter()
    geoms_np = W.batch_geometries(count, seed=4, nmin=64, nmax=max_edge)
    gs = [rd.Geometry(img, None, w.dx, 8) for img, _ in geoms_np]
    cat = rd.Geometry.concat(gs)
    n_active = cat.stats()["n_active"]
    log(f"batched stepping: {count} packings, {n_active} active voxels, indexed in {time.perf_counter() - t0:.1f}s")
    warm = 20
    with torch.cuda.stream(stream):
        sim = build_sim(rd, cat, w, "fp32", 16)
        sim.bind(stream=stream)
        sim.autotune(w.dt, 50)
        launch = sim.get_launch()
        secs_b, _, timing_b = time_steps(torch, sim, stream, w.dt, warm, steps)
        # each packing alone, same launch setting (kernel, order, steps per graph)
        secs_s = 0.0
        equal = True
        for i, g in enumerate(gs):
            s1 = build_sim(rd, g, w, "fp32", launch["graph_steps"])
            s1.bind(stream=stream)
            s1.set_launch(launch["graph_steps"], bool(launch["use_graph"]), bool(launch["xcd_map"]))
            s1.set_kernel(launch["kernel"], launch["wg_per_cu"])
            secs, _, _ = time_steps(torch, s1, stream, w.dt, warm, steps)
            secs_s += secs
            if i in (0, count // 2, count - 1):  # the same steps give the same bits
                for sp in range(len(w.species_D)):
                    equal = equal and bool(torch.equal(sim.get_part_field(sp, i), s1.get_field(sp)))
            del s1
        torch.cuda.synchronize()
        del sim
    per_b, per_s = secs_b / steps, secs_s / steps
    log(f"batched stepping: {per_b * 1e3:.3f} ms per step for all {count} in shared launches, "
        f"{per_s * 1e3:.3f} ms one by one ({per_s / per_b:.2f}x); parts == single runs: {equal}")
    return {
        "geometries": count,
        "n_active_voxels": n_active,
        "steps": steps,
        "launch": launch,
        "ms_per_step_batched": per_b * 1e3,
        "ms_per_step_one_by_one": per_s * 1e3,
        "updates_per_s_batched": n_active * steps / secs_b,
        "updates_per_s_one_by_one": n_active * steps / secs_s,
        "speedup": per_s / per_b,
        "timing_batched": timing_b,
        "parts_equal_single_runs": equal,
        "note": "HIP events around the timed steps of each run (warm-up and binding excluded)",
    }


def fused_form(torch, rd, W, stream, fused=16, size=512):
    """Several steps per cooperative launch against one launch per step (captured graphs),
    same kernel (column with the x-face exchange, XCD-aware order), on the 64^3 sphere
    packing (a small volume: 512 blocks) and the soil volume; FP32 with stochastic
    rounding.  Both runs take the same number of steps and must give the same bits."""
    out = {}
    for name in ("spheres64", "soil512"):
        w = W.workload(name)
        if name == "soil512":
            img = W.gaussian_random_field_volume(size, 12.0, 0.3, seed=w.seed)
            steps, warm = 2000, 64
        else:
            img, _ = W.workload_geometry(name)
            steps, warm = w.steps, 64
        g = rd.Geometry(img, None, w.dx, 8)
        n_active = g.stats()["n_active"]
        rec = {"n_active_voxels": n_active, "n_blocks": g.stats()["n_blocks"], "steps": steps,
               "kernel": "column_xch", "fused_steps": fused}
        fields = {}
        with torch.cuda.stream(stream):
            for t in (1, fused):
                sim = build_sim(rd, g, w, "fp32", fused)
                sim.set_kernel("column_xch", 8)
                sim.set_fused_steps(t)
                sim.bind(stream=stream)
                secs, _, timing = time_steps(torch, sim, stream, w.dt, warm, steps)
                key = "one_launch_per_step" if t == 1 else "fused"
                rec[key] = {"ms_per_step": secs / steps * 1e3, "updates_per_s": n_active * steps / secs,
                            "alg_GBps": 2 * 4 * len(w.species_D) * n_active * steps / secs / 1e9,
                            "timing": timing}
                fields[t] = [sim.get_field(sp).clone() for sp in range(len(w.species_D))]
                del sim
            torch.cuda.synchronize()
        rec["bitwise_equal"] = all(bool(torch.equal(a, b)) for a, b in zip(fields[1], fields[fused]))
        rec["speedup"] = rec["one_launch_per_step"]["ms_per_step"] / rec["fused"]["ms_per_step"]
        log(f"fused {name}: {rec['one_launch_per_step']['ms_per_step']:.4f} ms/step with one launch per step "
            f"(graphs), {rec['fused']['ms_per_step']:.4f} with {fused} steps per launch "
            f"({rec['speedup']:.2f}x); same bits: {rec['bitwise_equal']}")
        out[name] = rec
    return out


def steady_form(torch, rd, W, size, axes, forms, tol, stream, max_iters=200000, prec=6, crop_forms=None):
    """Tortuosity of the ceramic-foam volume (solid matrix of overlapping pore spheres
    r ~ U(10, 30), pore fraction 0.15) along the first `axes` axes by conjugate
    gradients, per storage type; with the full 1024^3 volume, the same solves on its
    256^3 corner crop are checked against the stored oracle tortuosity."""
    import numpy as np

    t0 = time.perf_counter()
    w = W.workload("foam1024")
    img, _ = W.workload_geometry("foam1024") if size == 1024 else \
        W.boolean_spheres(size, 0.15, 10.0, 30.0, seed=w.seed, active="solid")
    log(f"foam {size}^3 generated in {time.perf_counter() - t0:.1f}s")
    geom = rd.Geometry(img, None, 1.0, 8)
    st = geom.stats()
    crop = np.ascontiguousarray(img[:FOAM_CROP, :FOAM_CROP, :FOAM_CROP]) if size == 1024 else None
    del img
    out = {"workload": f"foam{size}", "n_active": st["n_active"], "n_blocks": st["n_blocks"],
           "fill": st["fill"], "tol": tol, "cg_precond_jacobi_steps": prec, "runs": []}
    for storage in forms:
        with torch.cuda.stream(stream):
            sim = rd.Sim(geom, storage)
            sim.add_species(1.0)
            sim.set_cg_precond(prec)
            sim.bind(features=rd.RD_WS_SOLVER, stream=stream)
            for axis in range(axes):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = sim.steady_state(axis, tol, max_iters)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
                vi = float(st["n_active"]) * r["iters"]
                out["runs"].append({"storage": storage, "axis": axis, "tau": r["tau"],
                                    "rel_residual": r["rel_residual"], "iters": r["iters"],
                                    "converged": r["converged"], "seconds": secs,
                                    "active_voxel_cg_iterations_per_s": vi / secs,
                                    "alg_GBps": vi * cg_words(prec) * (4 if storage == "fp32" else 2) / secs / 1e9})
                log(f"steady {storage} axis {axis}: tau {r['tau']:.5f}, rel {r['rel_residual']:.2e}, "
                    f"{r['iters']} it, {secs:.1f}s")
            del sim
            torch.cuda.empty_cache()
    if crop is not None:
        out["oracle_check"] = foam_crop_check(torch, rd, np, crop, crop_forms or forms, tol, stream, prec)
    return out


FOAM_CROP = 256
GOLDEN = os.path.join(HERE, "tests", "golden")


def _sha256(img):
    import hashlib

    return hashlib.sha256(img.tobytes()).hexdigest()


def foam_crop_check(torch, rd, np, crop, forms, tol, stream, prec=6):
    """Tortuosity along x of the 256^3 corner crop of the foam, per storage type, against
    the stored FP64 oracle value (oracle CG to 1e-12, written by
    tests/golden/make_goldens.py)."""
    path = os.path.join(GOLDEN, "foam_crop256_tau.json")
    if not os.path.exists(path):
        return None
    ref = json.load(open(path))
    if ref["sha256"] != _sha256(crop):
        log("foam crop differs from the stored one: no oracle check")
        return None
    tau_o = ref["axes"]["0"]["tau"]
    res = {"volume": "256^3 corner crop of the 1024^3 foam", "axis": 0, "oracle_tau": tau_o,
           "runs": []}
    geom = rd.Geometry(crop, None, 1.0, 8)
    for storage in forms:
        with torch.cuda.stream(stream):
            sim = rd.Sim(geom, storage)
            sim.add_species(1.0)
            sim.set_cg_precond(prec)
            sim.bind(features=rd.RD_WS_SOLVER, stream=stream)
            r = sim.steady_state(0, tol, 200000)
            del sim
        err = abs(r["tau"] - tau_o) / tau_o
        res["runs"].append({"storage": storage, "tau": r["tau"], "rel_err_vs_oracle": err,
                            "rel_residual": r["rel_residual"], "iters": r["iters"]})
        log(f"foam crop {storage}: tau {r['tau']:.10f} vs oracle {tau_o:.10f} (rel {err:.2e})")
    return res


def adjoint_form(torch, rd, W, stream):
    """Checkpointed adjoint on the 256^3 diffusion-decay packing (p = 0.5): the target is
    the final field of a run with D = 1, k = 0.01; the gradient of the L2 misfit of the
    run with D = 0.8, k = 0.02 (2000 steps, checkpoints every 100)."""
    w = W.workload("decay256")
    img, _ = W.workload_geometry("decay256")
    geom = rd.Geometry(img, None, w.dx, w.block_edge)
    st = geom.stats()
    n, k = w.steps, 100
    with torch.cuda.stream(stream):
        sim = rd.Sim(geom, "fp32")
        sim.add_species(1.0)
        sim.add_reaction(0, -1, 0.01)
        sim.set_dirichlet(0, 0, 1.0)
        sim.bind(features=rd.RD_WS_ADJOINT, checkpoint_slots=(n + k - 1) // k + k - 1, stream=stream)
        sim.step(w.dt, n)
        target = sim.get_field(0).clone()
        sim.set_species_D(0, w.species_D[0])
        sim.set_reaction_rate(0, 0.02)
        zero = torch.zeros_like(target)
        sim.set_field(0, zero)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(w.dt, n)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t0
        sim.set_field(0, zero)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, gD, gk = sim.adjoint(target, n, w.dt, k, seed_is_target=True)
        torch.cuda.synchronize()
        adj = time.perf_counter() - t0
    log(f"adjoint: forward {fwd * 1e3:.1f} ms, forward with checkpoints + recompute + backward "
        f"{adj * 1e3:.1f} ms")
    # the same run with the smooth D(phi) factor: dL/de per voxel as well
    with torch.cuda.stream(stream):
        del sim
        sim = rd.Sim(geom, "fp32")
        sim.add_species(w.species_D[0])
        sim.add_reaction(0, -1, 0.02)
        sim.set_dirichlet(0, 0, 1.0)
        sim.bind(features=rd.RD_WS_ADJOINT | rd.RD_WS_DIFFUSIVITY,
                 checkpoint_slots=(n + k - 1) // k + k - 1, stream=stream)
        phi = rd.sdf_from_image(torch.from_numpy(img).to("cuda"), 1.0, stream)
        sim.set_diffusivity_sdf(phi, *DIFF_PARS)
        sim.set_field(0, zero)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(w.dt, n)
        torch.cuda.synchronize()
        ffwd = time.perf_counter() - t0
        sim.set_field(0, zero)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        floss, fgD, fgk, ge = sim.adjoint_factor(target, n, w.dt, k, seed_is_target=True)
        torch.cuda.synchronize()
        fadj = time.perf_counter() - t0
        ge_norm = float(torch.linalg.vector_norm(ge))
    log(f"adjoint with a factor: forward {ffwd * 1e3:.1f} ms, adjoint with dL/de {fadj * 1e3:.1f} ms")
    factor = {"diffusivity": "e = %g + %g / (1 + exp(-(%g + %g phi)))" % DIFF_PARS,
              "forward_seconds": ffwd, "adjoint_seconds": fadj, "adjoint_over_forward": fadj / ffwd,
              "loss": floss, "dL_dD": fgD, "dL_drate": fgk, "dL_de_l2": ge_norm}
    res = {"workload": "decay256", "n_active": st["n_active"], "steps": n, "checkpoint_every": k,
           "forward_seconds": fwd, "adjoint_seconds": adj, "adjoint_over_forward": adj / fwd,
           "loss": loss, "dL_dD": gD, "dL_drate": gk, "factor": factor,
           "note": "adjoint_seconds: forward with checkpoints, recompute of each segment, "
                   "backward sweep; FP32 fields, FP64 gradient sums"}
    path = os.path.join(GOLDEN, "decay256_adjoint.json")
    if os.path.exists(path):
        ref = json.load(open(path))
        if ref["sha256"] == _sha256(img):
            res["oracle_check"] = {
                "oracle_dL_dD": ref["dL_dD"], "oracle_dL_drate": ref["dL_dk"],
                "central_difference_dL_dD": ref["fd"]["D"]["central"],
                "central_difference_dL_drate": ref["fd"]["k"]["central"],
                "rel_err_dL_dD": abs(gD - ref["dL_dD"]) / abs(ref["dL_dD"]),
                "rel_err_dL_drate": abs(gk - ref["dL_dk"]) / abs(ref["dL_dk"]),
                "note": "stored FP64 oracle adjoint and central differences (h = 1e-3) use the "
                        "oracle's FP64 target rounded to FP32; the bench's target is the same "
                        "run on the GPU in FP32, so the differences include that of the targets "
                        "(the parity test uses the oracle's target on both sides)"}
            log(f"adjoint vs stored oracle: dL/dD rel {res['oracle_check']['rel_err_dL_dD']:.2e}, "
                f"dL/dk rel {res['oracle_check']['rel_err_dL_drate']:.2e}")
    return res


# Smooth diffusivity of the inhomogeneous form: e = D_MIN + D_MAX / (1 + exp(-(G1 + G2 phi)))
# with phi the distance to the pore wall (voxels): 0.1 at the wall, 1.0 deep in the
# pores, the transition 1.5 voxels in and about a voxel wide.
DIFF_PARS = (0.1, 0.9, -6.0, 4.0)


def diffusivity_form(torch, rd, np, geom, img, w, n_active, steps, graph_steps, use_graph, stream):
    """FP32 steps of the soil volume with the smooth D(phi) factor (inhomogeneous step
    kernel), phi from the library's GPU distance transform.  Algorithmic bytes per
    launch: read + write of every species plus the 4-byte factor, per active voxel."""
    S = len(w.species_D)
    with torch.cuda.stream(stream):
        dimg = torch.from_numpy(img).to("cuda")
        rd.sdf_from_image(dimg, 1.0, stream)  # warm-up (first launches)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        phi = rd.sdf_from_image(dimg, 1.0, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sdf_ms = e0.elapsed_time(e1)
        log(f"diffusivity: signed distance of the {img.shape[0]}^3 image on the GPU in {sdf_ms:.1f} ms")
        sim = build_sim(rd, geom, w, "fp32", graph_steps, use_graph)
        sim.set_kernel("column_xch")
        sim.bind(features=rd.RD_WS_DIFFUSIVITY, stream=stream)
        sim.set_diffusivity_sdf(phi, *DIFF_PARS)
        del phi, dimg
        secs, wall, timing = time_steps(torch, sim, stream, w.dt, 50, steps)
        bal = [sim.balance(sp) for sp in range(S)]
        torch.cuda.synchronize()
    per = secs / steps
    alg = (2 * 4 * S + 4) * n_active
    res = {
        "kernel": f"k_step8e<float,{S},true>",
        "diffusivity": "e = %g + %g / (1 + exp(-(%g + %g phi))), phi = distance to the wall - 1/2"
                       % DIFF_PARS,
        "sdf_ms": sdf_ms,
        "steps": steps,
        "seconds": secs,
        "wall_seconds": wall,
        "ms_per_step": per * 1e3,
        "timing": timing,
        "updates_per_s": n_active * steps / secs,
        "alg_bytes_per_launch": alg,
        "alg_GBps": alg / per / 1e9,
        "frac_of_hbm_peak": alg / per / 1e9 / HBM_PEAK_GBS,
        "mass": [b["mass"] for b in bal],
        "inflow": [float(np.sum(b["inflow"])) for b in bal],
    }
    log(f"diffusivity: {per * 1e3:.4f} ms/step, {n_active * steps / secs:.3e} upd/s, "
        f"alg {alg / per / 1e9:.0f} GB/s")
    return res


def frap_tau(torch, rd, np, img, stream):
    """Simulated FRAP on one porous volume and on a free-space box of the same size:
    bleached central box of edge n/4, D = 1, dt = 0.1; D_eff from the least-squares fit,
    tau_d = 1 / D_eff, and the steady-state tortuosity of the same volume along x."""
    n = img.shape[0]
    q = max(1, n // 8)
    reg = (n // 2 - q, n // 2 + q) * 3
    x0, x1, y0, y1, z0, z1 = reg
    dt = 0.1
    # recovery time scale ~ (n/4)^2 / D: sample the porous run over ~ 1.2 of it
    t_end = 1.2 * (2 * q) ** 2
    sps = max(1, int(round(t_end / 60 / dt)))
    runs = {}
    t0 = time.perf_counter()
    for name, im, sp, ns in (("porous", img, sps, 60), ("free", np.ones_like(img), max(1, sps // 5), 300)):
        c0 = (im != 0).astype(np.float32)
        c0[z0:z1, y0:y1, x0:x1] = 0.0
        cinf = float(c0.sum()) / float((im != 0).sum())
        m_inf = cinf * float((im[z0:z1, y0:y1, x0:x1] != 0).sum())
        with torch.cuda.stream(stream):
            geom = rd.Geometry(im, None, 1.0, 8)
            sim = rd.Sim(geom, "fp32")
            sim.add_species(1.0)
            sim.bind(stream=stream)
            sim.set_field(0, torch.from_numpy(c0).to("cuda"))
            ts = time.perf_counter()
            curve = sim.frap_curve(0, reg, dt, sp, ns)
            secs = time.perf_counter() - ts
        runs[name] = {"curve": curve / m_inf, "seconds": secs, "steps": sp * ns, "samples": ns + 1,
                      "n_active": geom.stats()["n_active"], "dt_sample": sp * dt}
        del sim, geom
    por, free = runs["porous"], runs["free"]
    t = np.arange(por["samples"]) * por["dt_sample"]
    d_eff, rms = rd.frap_fit(t, por["curve"], free["dt_sample"], free["curve"], 1.0)
    wall = time.perf_counter() - t0
    with torch.cuda.stream(stream):
        geom = rd.Geometry(img, None, 1.0, 8)
        sim = rd.Sim(geom, "fp32")
        sim.add_species(1.0)
        sim.bind(features=rd.RD_WS_SOLVER, stream=stream)
        ts = time.perf_counter()
        ss = sim.steady_state(0, 1e-8, 100000)
        t_ss = time.perf_counter() - ts
        del sim, geom
    return {"n": n, "porosity": float((img != 0).mean()), "D_eff": d_eff, "tau_frap": 1.0 / d_eff,
            "fit_rms": rms, "tau_steady_x": ss["tau"], "steady_iterations": ss["iters"],
            "steady_seconds": t_ss, "frap_wall_seconds": wall, "porous_steps": por["steps"],
            "porous_seconds": por["seconds"],
            "porous_updates_per_s": por["n_active"] * por["steps"] / por["seconds"],
            "free_steps": free["steps"], "free_seconds": free["seconds"]}


def frap_form(torch, rd, np, W, n, stream):
    """FRAP tortuosity of an n^3 pore phase of overlapping balls (radii 4-8, porosity 0.5),
    then of the first eight packings of the batched workload, each beside its
    steady-state tortuosity along x."""
    img, _ = W.boolean_spheres(n, 0.5, 4.0, 8.0, seed=7)
    res = frap_tau(torch, rd, np, img, stream)
    res["volume"] = (f"{n}^3 pore phase of overlapping balls (radii 4-8, porosity 0.5), bleached "
                     f"central box of edge n/4, D = 1, dt = 0.1")
    log(f"frap: D_eff {res['D_eff']:.4f} tau {res['tau_frap']:.4f} (steady tau_x "
        f"{res['tau_steady_x']:.4f}); porous {res['porous_steps']} steps in {res['porous_seconds']:.2f}s")
    packs = []
    for im, info in W.batch_geometries(count=8):
        r = frap_tau(torch, rd, np, im, stream)
        packs.append({k: r[k] for k in ("n", "porosity", "tau_frap", "tau_steady_x", "fit_rms")})
        log(f"frap packing n={r['n']} porosity {r['porosity']:.3f}: tau_frap {r['tau_frap']:.4f} "
            f"tau_steady_x {r['tau_steady_x']:.4f}")
    res["batch_packings"] = packs
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the sparse-block stepper is "
              "not sharded across GPUs: the library runs on one GPU", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    import workloads as W
    from paper_2304_11165_amd import rd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.profile_form:
        stream = torch.cuda.Stream()
        if a.profile_form == "steady":
            rec = steady_form(torch, rd, W, a.steady_size, a.steady_axes,
                              [f for f in a.steady_forms.split(",") if f], a.steady_tol, stream,
                              a.steady_max_iters, a.cg_precond,
                              [f for f in a.steady_crop_forms.split(",") if f])
        elif a.profile_form == "batch":
            rec = batched_form(torch, rd, W, a.batch, a.batch_max_edge, stream, a.cg_precond)
        elif a.profile_form == "batch_steps":
            rec = batched_step_form(torch, rd, W, a.batch, a.batch_max_edge, a.batch_steps, stream)
        elif a.profile_form == "fused":
            rec = fused_form(torch, rd, W, stream, a.fused_steps, a.size)
        else:
            rec = adjoint_form(torch, rd, W, stream)
        print(json.dumps({"profile_form": a.profile_form, "record": rec}), flush=True)
        return
    w = W.workload("soil512")
    n = a.size
    t0 = time.perf_counter()
    img = W.gaussian_random_field_volume(n, 12.0, 0.3, seed=w.seed)
    log(f"geometry {n}^3 generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    geom = rd.Geometry(img, None, w.dx, w.block_edge)
    st = geom.stats()
    log(f"index built in {time.perf_counter() - t0:.1f}s: {st}")
    n_active, nb, fill = st["n_active"], st["n_blocks"], st["fill"]
    S = len(w.species_D)
    slots = nb * w.block_edge ** 3

    stream = torch.cuda.Stream()
    results, fields = {}, {}
    forms = [] if a.profile else [f for f in a.forms.split(",") if f]
    for storage in [a.profile_storage] if a.profile else ["fp32"] + forms:
        steps = a.steps if storage == "fp32" else min(a.steps, a.form_steps)
        warm = a.warmup
        layouts = ["blocks", "compact"] if a.layout == "auto" else [a.layout]
        if a.kernel in ("block", "persistent"):
            layouts = ["blocks"]  # the compact layout has only the column kernels
        with torch.cuda.stream(stream):
            cands = []
            for lay in layouts:
                sim = build_sim(rd, geom, w, storage, a.graph_steps, not a.no_graph)
                sim.set_layout(lay)
                sim.bind(stream=stream)
                if a.kernel != "auto":
                    sim.set_kernel(a.kernel)
                if a.xcd != "auto":
                    sim.set_launch(a.graph_steps, not a.no_graph, a.xcd == "1")
                cands.append(sim)
            tuned = a.kernel == "auto" or a.xcd == "auto"
            pick_ms = None
            if tuned and len(cands) > 1:
                best, pick_ms = rd.autotune_pick(cands, w.dt, 200)  # resets the fields
            else:
                best = 0
                if tuned:
                    cands[0].autotune(w.dt, 200)
            sim = cands[best]
            layout = layouts[best]
            del cands
            launch = sim.get_launch()
            launch["layout"] = layout
            if pick_ms is not None:
                launch["trial_ms_per_step"] = {lay: float(m) for lay, m in zip(layouts, pick_ms)}
            secs, wall, timing = time_steps(torch, sim, stream, w.dt, warm, steps)
            bal = [sim.balance(sp) for sp in range(S)]
            if storage != "fp32" or forms:
                fields[storage] = [sim.get_field(sp).float() for sp in range(S)]
            torch.cuda.synchronize()
        es = 4 if storage == "fp32" else 2
        alg_bytes = 2 * es * S * n_active
        if layout == "compact":  # active voxels + records, block bases and codes
            layout_bytes = 2 * es * S * n_active + nb * (32 + 128 + 4) + n_active
        else:  # whole blocks + records + codes
            layout_bytes = 2 * es * S * slots + nb * (32 + 128 + 512)
        per_step = secs / steps
        results[storage] = {
            "steps": steps,
            "warmup": warm,
            "seconds": secs,
            "wall_seconds": wall,
            "ms_per_step": per_step * 1e3,
            "timing": timing,
            "updates_per_s": n_active * steps / secs,
            "alg_GBps": alg_bytes / per_step / 1e9,
            "layout_GBps": layout_bytes / per_step / 1e9,
            "alg_bytes_per_launch": alg_bytes,
            "layout_bytes_per_launch": layout_bytes,
            "rounding": "stochastic",
            "launch": launch,
            "mass": [b["mass"] for b in bal],
            "inflow": [float(np.sum(b["inflow"])) for b in bal],
            "uptake": [b["uptake"] for b in bal],
        }
        log(f"{storage}: {per_step * 1e3:.4f} ms/step ({timing['ms_per_step_mean']:.4f} +- "
            f"{timing['ms_per_step_stderr']:.4f} over {timing['chunks']} chunks of "
            f"{timing['steps_per_chunk']}), {n_active * steps / secs:.3e} upd/s, "
            f"alg {alg_bytes / per_step / 1e9:.0f} GB/s, layout {layout_bytes / per_step / 1e9:.0f} GB/s")
        del sim

    # reduced-storage accuracy against an FP32-storage run of the same length (timed steps
    # and warm-up steps)
    for storage in forms:
        steps = results[storage]["steps"] + results[storage]["warmup"]
        with torch.cuda.stream(stream):
            ref = build_sim(rd, geom, w, "fp32", a.graph_steps)
            ref.bind(stream=stream)
            ref.step(w.dt, steps)
            errs = []
            for sp in range(S):
                r = ref.get_field(sp).float()
                d = fields[storage][sp] - r
                errs.append(float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(r)))
            torch.cuda.synchronize()
        results[storage]["rel_l2_vs_fp32_storage"] = errs
        del ref

    if a.profile and a.profile_storage != "fp32":
        print(json.dumps({"profile": results}), flush=True)
        return
    f32 = results["fp32"]
    kname = step_kernel_name(w.block_edge, f32["launch"], S)
    workload_name = f"soil{n}"
    traffic = load_traffic(a.traffic, kname, workload_name, f32["launch"]["xcd_map"])
    out = {
        "metric": METRIC,
        "value": f32["updates_per_s"],
        "unit": "active-voxel updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"soil-like {n}^3 Gaussian random field (corr. length 12, porosity 0.3), "
                        f"8^3 blocks, 2 species D=(1.0,0.4), A->B k=0.01, Robin on B k=0.05, "
                        f"c_A=1 on x=0, dt=0.1, FP32 storage (stochastic rounding)",
            "n_active_voxels": n_active,
            "n_blocks": nb,
            "fill": fill,
            "species": S,
            "steps_per_graph": f32["launch"]["graph_steps"],
            "launch": f32["launch"],
            "timed_as": f"{f32['timing']['chunks']} chunks of {f32['timing']['steps_per_chunk']} "
                        f"step(s), {f32['timing']['launches']}",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": f32["alg_GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": f32["alg_GBps"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": f32["alg_bytes_per_launch"],
            "layout_GBps": f32["layout_GBps"],
            "avg_launch_ms": f32["ms_per_step"],
            "avg_launch_ms_stderr": f32["timing"]["ms_per_step_stderr"],
        },
        "forms": results,
    }
    if a.batch > 0 and not a.profile:
        out["forms"]["batched"] = batched_form(torch, rd, W, a.batch, a.batch_max_edge, stream, a.cg_precond)
        if a.batch_steps > 0:
            out["forms"]["batched_steps"] = batched_step_form(torch, rd, W, a.batch, a.batch_max_edge,
                                                              a.batch_steps, stream)
    if a.fused_steps > 1 and not a.profile:
        out["forms"]["fused"] = fused_form(torch, rd, W, stream, a.fused_steps, a.size)
        log(f"batched: {out['forms']['batched']['active_voxel_cg_iterations_per_s']:.3e} "
            f"voxel-iterations/s")

    if a.steady_axes > 0 and not a.profile:
        out["forms"]["steady"] = steady_form(torch, rd, W, a.steady_size, a.steady_axes,
                                             [f for f in a.steady_forms.split(",") if f],
                                             a.steady_tol, stream, prec=a.cg_precond,
                                             crop_forms=[f for f in a.steady_crop_forms.split(",") if f])

    if a.diffusivity_steps > 0 and not a.profile:
        out["forms"]["diffusivity"] = diffusivity_form(torch, rd, np, geom, img, w, n_active,
                                                       a.diffusivity_steps, a.graph_steps,
                                                       not a.no_graph, stream)

    if a.frap_size > 0 and not a.profile:
        out["forms"]["frap"] = frap_form(torch, rd, np, W, a.frap_size, stream)

    if a.adjoint and not a.profile:
        out["forms"]["adjoint"] = adjoint_form(torch, rd, W, stream)

    if not a.no_cpu_baseline and not a.profile:
        out["cpu_baseline"] = cpu_baseline(img, w, n, n_active, a.cpu_steps, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img, w, n, n_active, cpu_steps, cpu_seconds):
    """The FP64 oracle on the host cores: three samples with every OpenMP thread (the
    median is the value), then one sample on a single thread."""
    import statistics

    import oracle

    prob = oracle.Problem(img, w.species_D, dx=w.dx, robin=w.robin, dirichlet=w.dirichlet,
                          reactions=w.reactions)
    threads = oracle.num_threads()
    c0 = prob.initial()
    prob.run(c0, w.dt, 1)  # page in
    done = cpu_steps
    if done <= 0:  # size a sample from two short runs (their difference drops the
        # per-call cost of copying the field in and out)
        t0 = time.perf_counter()
        prob.run(c0, w.dt, 2)
        t2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        prob.run(c0, w.dt, 6)
        t6 = time.perf_counter() - t0
        per = max((t6 - t2) / 4, 1e-6)
        done = max(2, min(5000, int((cpu_seconds - t2 + 2 * per) / per)))
    rates = []
    for _ in range(3):
        t0 = time.perf_counter()
        prob.run(c0, w.dt, done)
        rates.append(n_active * done / (time.perf_counter() - t0))
    oracle.set_num_threads(1)
    one = 2
    t0 = time.perf_counter()
    prob.run(c0, w.dt, one)
    rate1 = n_active * one / (time.perf_counter() - t0)
    oracle.set_num_threads(threads)
    res = {
        "value": statistics.median(rates),
        "unit": "active-voxel updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"median of 3 runs of {done} FP64 steps of the same {n}^3 two-species workload "
                  f"on the dense masked grid, {threads} OpenMP threads",
        "runs": rates,
        "value_single_thread": rate1,
        "single_thread_sample": f"{one} steps on one thread",
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }
    log(f"cpu oracle: {res['value']:.3e} upd/s on {threads} threads (runs "
        f"{', '.join(f'{r:.3e}' for r in rates)}), {rate1:.3e} on one thread; {res['cpu_model']}")
    return res


if __name__ == "__main__":
    main()
