"""Thin Python binding of librd.so (argument marshalling only).

Every computation happens in the HIP library; this module only converts NumPy /
torch objects into pointers and sizes, allocates the caller-owned device
workspace with torch, and passes torch's stream handle.  There is no fallback:
if librd.so is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2304_11165_amd.build.build() "
                      "(or __graft_entry__.build()) first")

# torch first: its HIP runtime (soname libamdhip64.so.7) is then the one librd.so
# binds to, so device pointers and stream handles from torch are valid in the
# library.  Loading librd.so first would bring in a second HIP runtime.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
i64, i32, u32, f64, ci = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
sz = ctypes.c_size_t

RD_OK = 0
STATUS = ["RD_OK", "RD_ERR_ARG", "RD_ERR_SHAPE", "RD_ERR_INCONSISTENT_SDF", "RD_ERR_UNSTABLE_DT",
          "RD_ERR_WORKSPACE", "RD_ERR_HIP", "RD_ERR_NONFINITE", "RD_ERR_NOT_CONVERGED",
          "RD_ERR_STATE"]
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2}
RD_WS_SOLVER = 1
RD_WS_ADJOINT = 2
RD_WS_DIFFUSIVITY = 4
# B = 8 step kernels, by number (column_lanes: compact layout only)
KERNELS = ("block", "persistent", "column", "column_xch", "column_lanes")

_SIGS = {
    "rd_status_string": ([ci], ctypes.c_char_p),
    "rd_last_error": ([], ctypes.c_char_p),
    "rd_geometry_create": ([P, P, i64, i64, i64, f64, ci, P], ci),
    "rd_geometry_stats": ([P, P, P, P, P], ci),
    "rd_geometry_export_index": ([P, P, P], ci),
    "rd_geometry_export_masks": ([P, P], ci),
    "rd_geometry_export_codes": ([P, P], ci),
    "rd_geometry_destroy": ([P], None),
    "rd_geometry_concat": ([P, ci, P], ci),
    "rd_geometry_parts": ([P], ci),
    "rd_geometry_part_info": ([P, ci, P, P, P, P], ci),
    "rd_sim_balance_part": ([P, ci, ci, P], ci),
    "rd_sim_set_fused_steps": ([P, ci], ci),
    "rd_sim_get_fused_steps": ([P, P], ci),
    "rd_sim_create": ([P, ci, P], ci),
    "rd_sim_add_species": ([P, f64, P], ci),
    "rd_sim_add_reaction": ([P, ci, ci, f64], ci),
    "rd_sim_set_robin": ([P, ci, f64], ci),
    "rd_sim_set_dirichlet": ([P, ci, ci, f64], ci),
    "rd_sim_clear_dirichlet": ([P, ci], ci),
    "rd_sim_set_launch": ([P, ci, ci, ci], ci),
    "rd_sim_set_kernel": ([P, ci, ci], ci),
    "rd_sim_set_rounding": ([P, ci, ctypes.c_uint64], ci),
    "rd_sim_workspace_bytes": ([P, u32, i64, P], ci),
    "rd_sim_bind": ([P, P, sz, u32, i64, P], ci),
    "rd_sim_set_field": ([P, ci, P], ci),
    "rd_sim_set_diffusivity": ([P, P], ci),
    "rd_sim_set_diffusivity_sdf": ([P, P, f64, f64, f64, f64], ci),
    "rd_sim_clear_diffusivity": ([P], ci),
    "rd_sim_set_sink": ([P, ci, f64], ci),
    "rd_sim_set_sink_band": ([P, P, f64, P], ci),
    "rd_sim_region_mass": ([P, ci, P, P], ci),
    "rd_sdf_scratch_bytes": ([i64, i64, i64, P], ci),
    "rd_sdf_from_image": ([P, i64, i64, i64, f64, P, P, ctypes.c_size_t, P], ci),
    "rd_sdf_from_image_static": ([P, i64, i64, i64, f64, P, P], ci),
    "rd_sim_set_layout": ([P, ci], ci),
    "rd_batch_set_launch": ([P, ci, ci], ci),
    "rd_batch_get_launch": ([P, P, P], ci),
    "rd_batch_set_cg_precond": ([P, ci], ci),
    "rd_sim_set_cg_precond": ([P, ci], ci),
    "rd_sim_frap_curve": ([P, ci, P, f64, i64, i64, P], ci),
    "rd_frap_fit": ([i64, P, P, i64, f64, P, f64, P, P], ci),
    "rd_sim_get_field": ([P, ci, P], ci),
    "rd_sim_step": ([P, f64, i64], ci),
    "rd_sim_steps_taken": ([P, P], ci),
    "rd_sim_reduce": ([P, ci, P, P, P], ci),
    "rd_sim_balance": ([P, ci, P], ci),
    "rd_sim_plane_flux": ([P, ci, ci, i64, P], ci),
    "rd_sim_steady_state": ([P, ci, f64, i64, P, P, P], ci),
    "rd_sim_adjoint": ([P, P, ci, i64, f64, ci, P, P, P], ci),
    "rd_sim_adjoint_factor": ([P, P, ci, i64, f64, ci, P, P, P, P], ci),
    "rd_sim_set_species_D": ([P, ci, f64], ci),
    "rd_sim_set_reaction_rate": ([P, ci, f64], ci),
    "rd_sim_destroy": ([P], None),
    "rd_sim_autotune": ([P, f64, i64, P], ci),
    "rd_sim_autotune_cached": ([P, f64, i64, ctypes.c_char_p, P, P], ci),
    "rd_autotune_pick": ([P, ci, f64, i64, P, P], ci),
    "rd_sim_get_launch": ([P, P, P, P, P, P], ci),
    "rd_batch_create": ([P, ci, ci, P], ci),
    "rd_batch_workspace_bytes": ([P, P], ci),
    "rd_batch_bind": ([P, P, sz, P], ci),
    "rd_batch_tortuosity": ([P, ci, f64, i64, P, P, P], ci),
    "rd_batch_autotune_pick": ([P, ci, ci, i64, P, P], ci),
    "rd_batch_destroy": ([P], None),
}

EXPORTED = sorted(_SIGS)

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)  # AttributeError here means the library lacks a declared symbol
    _f.argtypes = _args
    _f.restype = _res


class RDError(RuntimeError):
    def __init__(self, status, func):
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        detail = _lib.rd_last_error().decode()
        super().__init__(f"{func}: {self.name}: {detail}")


def _check(status, func):
    if status != RD_OK:
        raise RDError(status, func)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(P)


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# same-name functions
# ---------------------------------------------------------------------------

def rd_geometry_create(image, sdf=None, dx=1.0, block_edge=8):
    img = np.ascontiguousarray(image, dtype=np.uint8)
    if img.ndim != 3:
        raise ValueError("image must be (nz, ny, nx)")
    nz, ny, nx = img.shape
    s = None
    if sdf is not None:
        s = np.ascontiguousarray(sdf, dtype=np.float32)
        if s.shape != img.shape:
            raise ValueError("sdf shape differs from image")
    h = P()
    _check(_lib.rd_geometry_create(_np_ptr(img), _np_ptr(s), nx, ny, nz, float(dx),
                                   int(block_edge), ctypes.byref(h)), "rd_geometry_create")
    return h


def rd_geometry_stats(h):
    na, nb, por, fill = i64(), i64(), f64(), f64()
    _check(_lib.rd_geometry_stats(h, ctypes.byref(na), ctypes.byref(nb), ctypes.byref(por),
                                  ctypes.byref(fill)), "rd_geometry_stats")
    return na.value, nb.value, por.value, fill.value


def rd_geometry_export_index(h):
    nb = rd_geometry_stats(h)[1]
    ids = np.zeros(nb, dtype=np.int64)
    nbr = np.zeros((nb, 6), dtype=np.int32)
    _check(_lib.rd_geometry_export_index(h, _np_ptr(ids), _np_ptr(nbr)), "rd_geometry_export_index")
    return ids, nbr


def rd_geometry_export_masks(h, block_edge):
    nb = rd_geometry_stats(h)[1]
    words = max(1, block_edge ** 3 // 64)
    m = np.zeros((nb, words), dtype=np.uint64)
    _check(_lib.rd_geometry_export_masks(h, _np_ptr(m)), "rd_geometry_export_masks")
    return m


def rd_geometry_destroy(h):
    _lib.rd_geometry_destroy(h)


# ---------------------------------------------------------------------------
# objects
# ---------------------------------------------------------------------------

class Geometry:
    """Active-block index of a voxel image (host only)."""

    def __init__(self, image, sdf=None, dx=1.0, block_edge=8):
        self.shape = tuple(int(v) for v in np.asarray(image).shape)
        self.dx = float(dx)
        self.block_edge = int(block_edge)
        self.handle = rd_geometry_create(image, sdf, dx, block_edge)

    def stats(self):
        na, nb, por, fill = rd_geometry_stats(self.handle)
        return {"n_active": na, "n_blocks": nb, "porosity": por, "fill": fill}

    def export_index(self):
        return rd_geometry_export_index(self.handle)

    def export_masks(self):
        return rd_geometry_export_masks(self.handle, self.block_edge)

    def export_codes(self):
        nb = rd_geometry_stats(self.handle)[1]
        c = np.zeros((nb, self.block_edge ** 3), dtype=np.uint8)
        _check(_lib.rd_geometry_export_codes(self.handle, _np_ptr(c)), "rd_geometry_export_codes")
        return c

    @classmethod
    def concat(cls, parts):
        """One geometry holding several (rd_geometry_concat): a Sim on it steps every part
        in the same launches; its dense fields hold the parts' boxes one after another
        (`shape` is (1, 1, total voxels); `parts()` gives each part's box and offset)."""
        parts = list(parts)
        arr = (ctypes.c_void_p * len(parts))(*[p.handle for p in parts])
        h = ctypes.c_void_p()
        _check(_lib.rd_geometry_concat(arr, len(parts), ctypes.byref(h)), "rd_geometry_concat")
        g = cls.__new__(cls)
        g.handle = h.value
        g.dx = parts[0].dx
        g.block_edge = parts[0].block_edge
        g.shape = (1, 1, int(sum(int(np.prod(p.shape)) for p in parts)))
        return g

    def parts(self):
        """[{shape, dense_offset, first_block, n_blocks}] per part (one for a plain geometry)."""
        out = []
        for i in range(_lib.rd_geometry_parts(self.handle)):
            shp = np.zeros(3, dtype=np.int64)
            off, b0, nb = i64(), i64(), i64()
            _check(_lib.rd_geometry_part_info(self.handle, i, _np_ptr(shp), ctypes.byref(off), ctypes.byref(b0),
                                              ctypes.byref(nb)), "rd_geometry_part_info")
            out.append({"shape": tuple(int(v) for v in shp), "dense_offset": off.value,
                        "first_block": b0.value, "n_blocks": nb.value})
        return out

    def __del__(self, _destroy=_lib.rd_geometry_destroy):
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


class Sim:
    """A reaction-diffusion simulation on one geometry (device work via librd)."""

    def __init__(self, geometry, storage="fp32"):
        self.geometry = geometry
        self.storage = storage
        self.handle = P()
        _check(_lib.rd_sim_create(geometry.handle, STORAGE[storage], ctypes.byref(self.handle)),
               "rd_sim_create")
        self.n_species = 0
        self.workspace = None
        self.stream = None

    # set-up ------------------------------------------------------------------
    def add_species(self, D):
        sid = ci()
        _check(_lib.rd_sim_add_species(self.handle, float(D), ctypes.byref(sid)), "rd_sim_add_species")
        self.n_species += 1
        return sid.value

    def add_reaction(self, src, dst, rate):
        _check(_lib.rd_sim_add_reaction(self.handle, int(src), int(dst), float(rate)),
               "rd_sim_add_reaction")

    def set_robin(self, species, k):
        _check(_lib.rd_sim_set_robin(self.handle, int(species), float(k)), "rd_sim_set_robin")

    def set_dirichlet(self, species, face, value):
        _check(_lib.rd_sim_set_dirichlet(self.handle, int(species), int(face), float(value)),
               "rd_sim_set_dirichlet")

    def clear_dirichlet(self, species):
        _check(_lib.rd_sim_clear_dirichlet(self.handle, int(species)), "rd_sim_clear_dirichlet")

    def set_launch(self, graph_steps=32, use_graph=True, xcd_map=False):
        _check(_lib.rd_sim_set_launch(self.handle, int(graph_steps), int(bool(use_graph)),
                                      int(bool(xcd_map))), "rd_sim_set_launch")

    def autotune(self, dt, trial_steps=200, cache_path=None):
        """Pick the fastest launch configuration; returns ms/step.  Without a cache the
        trials reset the fields; with `cache_path` a stored result for the same GPU,
        storage, species and geometry is applied without trials (see
        rd_sim_autotune_cached), else the trials run and are appended to the file."""
        ms = f64()
        if cache_path is None:
            _check(_lib.rd_sim_autotune(self.handle, float(dt), int(trial_steps), ctypes.byref(ms)),
                   "rd_sim_autotune")
            return ms.value
        hit = ci()
        _check(_lib.rd_sim_autotune_cached(self.handle, float(dt), int(trial_steps),
                                           os.fsencode(str(cache_path)), ctypes.byref(hit),
                                           ctypes.byref(ms)), "rd_sim_autotune_cached")
        self.last_tune_from_cache = bool(hit.value)
        return ms.value

    def get_launch(self):
        vals = [ci() for _ in range(5)]
        _check(_lib.rd_sim_get_launch(self.handle, *[ctypes.byref(v) for v in vals]),
               "rd_sim_get_launch")
        keys = ("graph_steps", "use_graph", "xcd_map", "kernel", "wg_per_cu")
        out = {k: v.value for k, v in zip(keys, vals)}
        out["kernel"] = KERNELS[out["kernel"]]
        return out

    def set_layout(self, layout="blocks"):
        """Field layout in HBM: "blocks" (every slot of the stored blocks) or "compact"
        (only the active voxels); before bind."""
        _check(_lib.rd_sim_set_layout(self.handle, {"blocks": 0, "compact": 1}[layout]),
               "rd_sim_set_layout")
        return self

    def set_kernel(self, kernel="block", wg_per_cu=8):
        """B = 8 step kernel: "block" (one workgroup per block), "persistent",
        "column" (one wave per block, z-columns) or "column_xch" (column with x faces
        exchanged inside the workgroup); or its number 0..3."""
        k = KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
        _check(_lib.rd_sim_set_kernel(self.handle, k, int(wg_per_cu)), "rd_sim_set_kernel")

    def set_rounding(self, stochastic, seed=0):
        _check(_lib.rd_sim_set_rounding(self.handle, int(bool(stochastic)), int(seed)),
               "rd_sim_set_rounding")

    def workspace_bytes(self, features=0, checkpoint_slots=0):
        n = sz()
        _check(_lib.rd_sim_workspace_bytes(self.handle, int(features), int(checkpoint_slots),
                                           ctypes.byref(n)), "rd_sim_workspace_bytes")
        return n.value

    def bind(self, features=0, checkpoint_slots=0, device="cuda", stream=None):
        import torch

        nbytes = self.workspace_bytes(features, checkpoint_slots)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.rd_sim_bind(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                self.workspace.numel(), int(features), int(checkpoint_slots),
                                _stream_handle(self.stream)), "rd_sim_bind")
        return self

    # fields ------------------------------------------------------------------
    def set_field(self, species, dense):
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(dense, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        _check(_lib.rd_sim_set_field(self.handle, int(species), ctypes.c_void_p(t.data_ptr())),
               "rd_sim_set_field")
        self._keep = t  # lives until the stream has consumed it
        return self

    def set_diffusivity(self, dense):
        """Per-voxel diffusivity factor e (dense (nz, ny, nx)): species s then diffuses
        with D_s * e, the mean of the two voxels' coefficients on each face.  Needs a
        bind with RD_WS_DIFFUSIVITY.  Synchronises."""
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(dense, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        _check(_lib.rd_sim_set_diffusivity(self.handle, ctypes.c_void_p(t.data_ptr())),
               "rd_sim_set_diffusivity")
        return self

    def set_diffusivity_sdf(self, sdf, d_min, d_max, gamma1, gamma2):
        """e = d_min + d_max / (1 + exp(-(gamma1 + gamma2 phi))) from a dense signed
        distance phi, evaluated on the GPU.  Synchronises."""
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(sdf, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        _check(_lib.rd_sim_set_diffusivity_sdf(self.handle, ctypes.c_void_p(t.data_ptr()),
                                               float(d_min), float(d_max), float(gamma1),
                                               float(gamma2)),
               "rd_sim_set_diffusivity_sdf")
        return self

    def region_mass(self, species, region):
        """FP64 mass of `species` over the active voxels of region (x0, x1, y0, y1, z0, z1)."""
        reg = np.ascontiguousarray(region, dtype=np.int64)
        m = f64()
        _check(_lib.rd_sim_region_mass(self.handle, int(species), _np_ptr(reg), ctypes.byref(m)),
               "rd_sim_region_mass")
        return m.value

    def frap_curve(self, species, region, dt, steps_per_sample, n_samples):
        """Region mass at k * steps_per_sample steps, k = 0..n_samples (steps are taken)."""
        reg = np.ascontiguousarray(region, dtype=np.int64)
        out = np.zeros(int(n_samples) + 1)
        _check(_lib.rd_sim_frap_curve(self.handle, int(species), _np_ptr(reg), float(dt),
                                      int(steps_per_sample), int(n_samples), _np_ptr(out)),
               "rd_sim_frap_curve")
        return out

    def set_sink(self, species, rate):
        """Volumetric sink rate of a species on the near-surface band."""
        _check(_lib.rd_sim_set_sink(self.handle, int(species), float(rate)), "rd_sim_set_sink")
        return self

    def set_sink_band(self, phi, band):
        """Mark the active voxels with phi < band as the sink band; returns their number."""
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(phi, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        n = i64()
        _check(_lib.rd_sim_set_sink_band(self.handle, ctypes.c_void_p(t.data_ptr()), float(band),
                                         ctypes.byref(n)), "rd_sim_set_sink_band")
        return n.value

    def clear_diffusivity(self):
        _check(_lib.rd_sim_clear_diffusivity(self.handle), "rd_sim_clear_diffusivity")
        return self

    def get_field(self, species, out=None):
        import torch

        nz, ny, nx = self.geometry.shape
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.workspace.device)
        _check(_lib.rd_sim_get_field(self.handle, int(species), ctypes.c_void_p(out.data_ptr())),
               "rd_sim_get_field")
        return out

    # time stepping --------------------------------------------------------------
    def set_fused_steps(self, steps):
        """Steps per cooperative launch (1: one launch per step); 8^3 blocks, block layout,
        column kernels, constant D (others keep one launch per step)."""
        _check(_lib.rd_sim_set_fused_steps(self.handle, int(steps)), "rd_sim_set_fused_steps")
        return self

    def get_fused_steps(self):
        n = ctypes.c_int()
        _check(_lib.rd_sim_get_fused_steps(self.handle, ctypes.byref(n)), "rd_sim_get_fused_steps")
        return n.value

    def step(self, dt, n_steps=1):
        _check(_lib.rd_sim_step(self.handle, float(dt), int(n_steps)), "rd_sim_step")
        return self

    def steps_taken(self):
        n = i64()
        _check(_lib.rd_sim_steps_taken(self.handle, ctypes.byref(n)), "rd_sim_steps_taken")
        return n.value

    def reduce(self, species):
        m, f, r = f64(), f64(), f64()
        _check(_lib.rd_sim_reduce(self.handle, int(species), ctypes.byref(m), ctypes.byref(f),
                                  ctypes.byref(r)), "rd_sim_reduce")
        return m.value, f.value, r.value

    def balance(self, species, part=None):
        """FP64 balance terms of `species`; `part`: only that part of a concatenated
        geometry."""
        out = np.zeros(9)
        if part is None:
            _check(_lib.rd_sim_balance(self.handle, int(species), _np_ptr(out)), "rd_sim_balance")
        else:
            _check(_lib.rd_sim_balance_part(self.handle, int(species), int(part), _np_ptr(out)),
                   "rd_sim_balance_part")
        return {"mass": out[0], "inflow": out[1:7].copy(), "uptake": out[7], "react": out[8]}

    def get_part_field(self, species, part):
        """Species `species` of part `part` of a concatenated geometry, (nz, ny, nx)."""
        info = self.geometry.parts()[part]
        n = int(np.prod(info["shape"]))
        flat = self.get_field(species).reshape(-1)
        return flat[info["dense_offset"]:info["dense_offset"] + n].reshape(info["shape"])

    def plane_flux(self, species, axis, i0):
        """FP64 diffusive flux of `species` through the plane between i0 and i0 + 1 along
        `axis` (0 x, 1 y, 2 z), positive towards +axis."""
        q = f64()
        _check(_lib.rd_sim_plane_flux(self.handle, int(species), int(axis), int(i0), ctypes.byref(q)),
               "rd_sim_plane_flux")
        return q.value

    def steady_state(self, axis, rel_tol=1e-8, max_iters=100000):
        tau, rel, it = f64(), f64(), i64()
        st = _lib.rd_sim_steady_state(self.handle, int(axis), float(rel_tol), int(max_iters),
                                      ctypes.byref(tau), ctypes.byref(rel), ctypes.byref(it))
        if st not in (RD_OK, 8):  # RD_ERR_NOT_CONVERGED still returns the values reached
            _check(st, "rd_sim_steady_state")
        return {"tau": tau.value, "rel_residual": rel.value, "iters": it.value,
                "converged": st == RD_OK}

    def set_cg_precond(self, jacobi_steps):
        """Jacobi steps of the steady-state CG's block preconditioner (0: plain CG)."""
        _check(_lib.rd_sim_set_cg_precond(self.handle, int(jacobi_steps)), "rd_sim_set_cg_precond")

    def set_species_D(self, species, D):
        _check(_lib.rd_sim_set_species_D(self.handle, int(species), float(D)), "rd_sim_set_species_D")

    def set_reaction_rate(self, index, rate):
        _check(_lib.rd_sim_set_reaction_rate(self.handle, int(index), float(rate)),
               "rd_sim_set_reaction_rate")

    def adjoint(self, seed, n_steps, dt, checkpoint_every, seed_is_target=True):
        """(loss, dL/dD, dL/dk) of the run from the current field.  seed: target field
        c* (seed_is_target) or dL/dc^N."""
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(seed, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        L, gD, gk = f64(), f64(), f64()
        _check(_lib.rd_sim_adjoint(self.handle, ctypes.c_void_p(t.data_ptr()),
                                   0 if seed_is_target else 1, int(n_steps), float(dt),
                                   int(checkpoint_every), ctypes.byref(L), ctypes.byref(gD),
                                   ctypes.byref(gk)), "rd_sim_adjoint")
        return L.value, gD.value, gk.value

    def adjoint_factor(self, seed, n_steps, dt, checkpoint_every, seed_is_target=True):
        """(loss, dL/dD, dL/dk, dL/de) with a diffusivity factor set; dL/de is a float64
        (nz, ny, nx) tensor on the GPU."""
        import torch

        nz, ny, nx = self.geometry.shape
        t = torch.as_tensor(seed, dtype=torch.float32, device=self.workspace.device)
        t = t.reshape(nz, ny, nx).contiguous()
        ge = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.workspace.device)
        L, gD, gk = f64(), f64(), f64()
        _check(_lib.rd_sim_adjoint_factor(self.handle, ctypes.c_void_p(t.data_ptr()),
                                          0 if seed_is_target else 1, int(n_steps), float(dt),
                                          int(checkpoint_every), ctypes.byref(L), ctypes.byref(gD),
                                          ctypes.byref(gk), ctypes.c_void_p(ge.data_ptr())),
               "rd_sim_adjoint_factor")
        return L.value, gD.value, gk.value, ge

    def __del__(self, _destroy=_lib.rd_sim_destroy):
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


class Batch:
    """Many geometries stepped together (single species, pure diffusion)."""

    def __init__(self, geometries, storage="fp32"):
        self.geometries = list(geometries)
        arr = (P * len(self.geometries))(*[g.handle for g in self.geometries])
        self._arr = arr
        self.handle = P()
        _check(_lib.rd_batch_create(arr, len(self.geometries), STORAGE[storage],
                                    ctypes.byref(self.handle)), "rd_batch_create")
        self.workspace = None

    def bind(self, device="cuda", stream=None):
        import torch

        n = sz()
        _check(_lib.rd_batch_workspace_bytes(self.handle, ctypes.byref(n)), "rd_batch_workspace_bytes")
        self.workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.rd_batch_bind(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                  self.workspace.numel(), _stream_handle(self.stream)),
               "rd_batch_bind")
        return self

    def set_cg_precond(self, jacobi_steps):
        _check(_lib.rd_batch_set_cg_precond(self.handle, int(jacobi_steps)), "rd_batch_set_cg_precond")

    def set_launch(self, iters_per_check=25, use_graph=True):
        _check(_lib.rd_batch_set_launch(self.handle, int(iters_per_check), 1 if use_graph else 0),
               "rd_batch_set_launch")
        return self

    def get_launch(self):
        it, gr = ci(), ci()
        _check(_lib.rd_batch_get_launch(self.handle, ctypes.byref(it), ctypes.byref(gr)),
               "rd_batch_get_launch")
        return {"iters_per_check": it.value, "use_graph": gr.value}

    def tortuosity(self, axis=0, rel_tol=1e-8, max_iters=100000):
        n = len(self.geometries)
        tau, rel, it = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int64)
        st = _lib.rd_batch_tortuosity(self.handle, int(axis), float(rel_tol), int(max_iters),
                                      _np_ptr(tau), _np_ptr(rel), _np_ptr(it))
        if st not in (RD_OK, 8):
            _check(st, "rd_batch_tortuosity")
        return tau, rel, it

    def __del__(self, _destroy=_lib.rd_batch_destroy):
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


def autotune_pick(sims, dt, trial_steps=200):
    """Autotune each bound candidate Sim (e.g. the same image with 4^3 and 8^3 blocks)
    and return (index of the fastest, ms per step of each)."""
    arr = (P * len(sims))(*[s.handle for s in sims])
    best = ci()
    ms = np.zeros(len(sims))
    _check(_lib.rd_autotune_pick(arr, len(sims), float(dt), int(trial_steps), ctypes.byref(best),
                                 _np_ptr(ms)), "rd_autotune_pick")
    return best.value, ms


def batch_autotune_pick(batches, axis=0, trial_iters=50):
    """Time trial_iters CG iterations of each bound candidate Batch (the same geometries
    indexed with 4^3 and 8^3 blocks, say) and return (index of the fastest, ms per
    iteration of each)."""
    arr = (P * len(batches))(*[b.handle for b in batches])
    best = ci()
    ms = np.zeros(len(batches))
    _check(_lib.rd_batch_autotune_pick(arr, len(batches), int(axis), int(trial_iters), ctypes.byref(best),
                                       _np_ptr(ms)), "rd_batch_autotune_pick")
    return best.value, ms


class DiffusionDecay(torch.autograd.Function):
    """c^N = FTCS^n(c^0; D, k) for a single-species diffusion-decay simulation, with
    gradients with respect to the scalars D and k from the library's checkpointed
    adjoint (rd_sim_adjoint, seed = dL/dc^N).

    Usage: ``cN = DiffusionDecay.apply(D, k, sim, c0, n_steps, dt, checkpoint_every)``
    with D, k 0-dim float64 tensors, sim a bound single-species Sim whose reaction 0
    is the decay, c0 a dense float32 device field."""

    @staticmethod
    def forward(ctx, D, k, sim, c0, n_steps, dt, checkpoint_every):
        sim.set_species_D(0, float(D))
        sim.set_reaction_rate(0, float(k))
        sim.set_field(0, c0)
        sim.step(dt, n_steps)
        out = sim.get_field(0)
        ctx.sim, ctx.c0, ctx.n, ctx.dt, ctx.k = sim, c0, n_steps, dt, checkpoint_every
        ctx.params = (float(D), float(k))
        return out

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        sim.set_species_D(0, ctx.params[0])
        sim.set_reaction_rate(0, ctx.params[1])
        sim.set_field(0, ctx.c0)
        _, gD, gk = sim.adjoint(g.float().contiguous(), ctx.n, ctx.dt, ctx.k, seed_is_target=False)
        dev = g.device
        return (torch.tensor(gD, dtype=torch.float64, device=dev),
                torch.tensor(gk, dtype=torch.float64, device=dev), None, None, None, None, None)


def frap_fit(t, f, ds, g, D_ref):
    """(D_eff, rms): the free-space coefficient whose recovery g(t D / D_ref) (g sampled
    at j * ds for D_ref) best fits f(t) in least squares (host computation)."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    d, r = f64(), f64()
    _check(_lib.rd_frap_fit(len(t), _np_ptr(t), _np_ptr(f), len(g), float(ds), _np_ptr(g),
                            float(D_ref), ctypes.byref(d), ctypes.byref(r)), "rd_frap_fit")
    return d.value, r.value


def sdf_from_image(image, dx=1.0, stream=None):
    """Signed distance (float32 (nz, ny, nx) tensor on the image's GPU) of a uint8 voxel
    image by the library's exact distance transform: (distance to the other phase - 1/2)
    dx, positive on active voxels."""
    import torch

    img = torch.as_tensor(image, dtype=torch.uint8)
    if not img.is_cuda:
        img = img.to("cuda")
    img = img.contiguous()
    nz, ny, nx = img.shape
    n = ctypes.c_size_t()
    _check(_lib.rd_sdf_scratch_bytes(nx, ny, nz, ctypes.byref(n)), "rd_sdf_scratch_bytes")
    scratch = torch.empty(max(n.value, 256), dtype=torch.uint8, device=img.device)
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device=img.device)
    st = stream if stream is not None else torch.cuda.current_stream(img.device)
    _check(_lib.rd_sdf_from_image(ctypes.c_void_p(img.data_ptr()), nx, ny, nz, float(dx),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(scratch.data_ptr()),
                                  scratch.numel(), _stream_handle(st)), "rd_sdf_from_image")
    # the allocator must not hand these out again before the stream has used them
    for t in (img, scratch, out):
        t.record_stream(st)
    return out


def sdf_from_image_static(image, out, dx=1.0, stream=None):
    """rd_sdf_from_image_static: the signed distance of a uint8 (nz, ny, nx) device image
    into the caller's float32 device tensor `out`, with the library's fixed per-GPU
    scratch (no allocation in the library; volumes up to 64 MiB of scratch, 20 bytes per
    voxel).  Calls on one GPU share that scratch: overlapping calls race."""
    import torch

    assert image.is_cuda and image.dtype == torch.uint8 and image.is_contiguous()
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
    assert tuple(out.shape) == tuple(image.shape)
    nz, ny, nx = image.shape
    st = stream if stream is not None else torch.cuda.current_stream(image.device)
    _check(_lib.rd_sdf_from_image_static(ctypes.c_void_p(image.data_ptr()), nx, ny, nz, float(dx),
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(st)),
           "rd_sdf_from_image_static")
    return out
