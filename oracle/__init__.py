"""Plain FP64 CPU oracle for sparse-grid reaction-diffusion (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2304_11165_amd``) and never imports it.

The arithmetic lives in ``rd_oracle.c`` (dense masked grid, FP64, loops written
as the definitions).  This module adds the ctypes marshalling, the active-block
index as an independent NumPy scan, and the tortuosity formula.

Paper: Stark & Sbalzarini, arXiv 2304.11165.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FACES = {"-x": 0, "+x": 1, "-y": 2, "+y": 3, "-z": 4, "+z": 5}


def build(force=True):
    """Compile rd_oracle.c into liboracle.so with gcc (-O3, OpenMP, no -march so the
    library also runs on a different host CPU)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, f64, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.orc_ftcs_run.argtypes = [i64, i64, i64, f64, P, ci, P, P, P, ci, P, P, P, P, f64, i64, P, P]
    lib.orc_ftcs_run.restype = ci
    lib.orc_balance.argtypes = [i64, i64, i64, f64, P, ci, P, P, P, ci, P, P, P, P, ci, P, P, P, P]
    lib.orc_balance.restype = ci
    lib.orc_ftcs_run_ext.argtypes = [i64, i64, i64, f64, P, ci, P, P, P, ci, P, P, P, P, P, P, P,
                                     f64, i64, P, P]
    lib.orc_ftcs_run_ext.restype = ci
    lib.orc_balance_ext.argtypes = [i64, i64, i64, f64, P, ci, P, P, P, ci, P, P, P, P, P, P, P, ci,
                                    P, P, P, P]
    lib.orc_balance_ext.restype = ci
    lib.orc_smooth_diffusivity.argtypes = [i64, P, f64, f64, f64, f64, P]
    lib.orc_smooth_diffusivity.restype = None
    lib.orc_plane_flux.argtypes = [i64, i64, i64, f64, P, f64, P, ci, i64]
    lib.orc_plane_flux.restype = f64
    lib.orc_plane_flux_eps.argtypes = [i64, i64, i64, f64, P, f64, P, P, ci, i64]
    lib.orc_plane_flux_eps.restype = f64
    lib.orc_steady_jacobi.argtypes = [i64, i64, i64, P, P, P, f64, i64, i64, P, P]
    lib.orc_steady_jacobi.restype = ci
    lib.orc_steady_cg.argtypes = [i64, i64, i64, P, P, P, f64, i64, P, P]
    lib.orc_steady_cg.restype = ci
    lib.orc_adjoint_decay.argtypes = [i64, i64, i64, f64, P, P, f64, f64, f64, i64, i64, P, P,
                                      P, P, P, P]
    lib.orc_adjoint_decay.restype = ci
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ci
    lib.orc_set_num_threads.argtypes = [ci]
    lib.orc_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads():
    return int(_load().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


class Problem:
    """A reaction-diffusion problem on a dense masked grid.

    image     uint8 (nz, ny, nx), 1 = active voxel (phi > 0)
    D         per-species diffusion coefficients
    robin     {species: k_R} wall uptake
    dirichlet {(species, face): value}; face 0..5 = -x,+x,-y,+y,-z,+z
    reactions [(from, to, rate)], to = -1 for decay
    """

    def __init__(self, image, D, dx=1.0, robin=None, dirichlet=None, reactions=None, eps=None,
                 sink=None, sink_mask=None):
        self.image = np.ascontiguousarray(image, dtype=np.uint8)
        # volumetric sink: rate sink[s] on the voxels where sink_mask is set
        self.sink_k = None
        self.sink_mask = None
        if sink:
            self.sink_k = np.zeros(len(np.atleast_1d(D)))
            for s, k in sink.items():
                self.sink_k[s] = k
            self.sink_mask = np.ascontiguousarray(np.asarray(sink_mask).reshape(self.image.shape),
                                                  dtype=np.uint8)
        # per-voxel diffusivity factor: D of species s at voxel p is D[s] * eps[p]
        self.eps = None if eps is None else np.ascontiguousarray(
            np.asarray(eps, dtype=np.float64).reshape(self.image.shape))
        assert self.image.ndim == 3
        self.nz, self.ny, self.nx = self.image.shape
        self.N = self.image.size
        self.dx = float(dx)
        self.D = np.ascontiguousarray(np.asarray(D, dtype=np.float64).ravel())
        self.S = len(self.D)
        self.robin = np.zeros(self.S)
        for s, k in (robin or {}).items():
            self.robin[s] = k
        self.dir_face = np.zeros((self.S, 6), dtype=np.uint8)
        self.dir_value = {}
        for (s, f), v in (dirichlet or {}).items():
            self.dir_face[s, f] = 1
            self.dir_value[(s, f)] = float(v)
        reactions = reactions or []
        self.r_from = np.array([r[0] for r in reactions], dtype=np.int32)
        self.r_to = np.array([r[1] for r in reactions], dtype=np.int32)
        self.r_rate = np.array([r[2] for r in reactions], dtype=np.float64)

    # -- helpers -----------------------------------------------------------
    def face_plane(self, f):
        """Boolean (nz,ny,nx) mask of the box-face plane f."""
        m = np.zeros(self.image.shape, dtype=bool)
        sl = [slice(None)] * 3
        axis = 2 - f // 2  # f 0,1 -> x (array axis 2)
        sl[axis] = 0 if f % 2 == 0 else self.image.shape[axis] - 1
        m[tuple(sl)] = True
        return m

    def dirichlet_mask(self, s):
        m = np.zeros(self.image.shape, dtype=bool)
        for f in range(6):
            if self.dir_face[s, f]:
                m |= self.face_plane(f)
        return m & (self.image != 0)

    def free_mask(self, s):
        return (self.image != 0) & ~self.dirichlet_mask(s)

    def apply_dirichlet(self, c):
        """Zero inactive voxels and write the Dirichlet values (in face order, the
        highest flagged face wins on shared edges)."""
        c = np.array(c, dtype=np.float64, copy=True).reshape(self.S, self.nz, self.ny, self.nx)
        c[:, self.image == 0] = 0.0
        for (s, f), v in sorted(self.dir_value.items()):
            m = self.face_plane(f) & (self.image != 0)
            c[s][m] = v
        return c

    def initial(self, fill=0.0):
        return self.apply_dirichlet(np.full((self.S, self.nz, self.ny, self.nx), fill))

    # -- oracle calls ------------------------------------------------------
    def run(self, c, dt, nsteps, source=None):
        """FTCS steps on a copy of c (S,nz,ny,nx) float64; returns the new field."""
        lib = _load()
        c = np.ascontiguousarray(np.array(c, dtype=np.float64, copy=True).reshape(
            self.S, self.nz, self.ny, self.nx))
        src = None
        if source is not None:
            src = np.ascontiguousarray(np.asarray(source, dtype=np.float64).reshape(c.shape))
        rc = lib.orc_ftcs_run_ext(self.nx, self.ny, self.nz, self.dx, _ptr(self.image), self.S,
                                  _ptr(self.D), _ptr(self.robin), _ptr(self.dir_face),
                                  len(self.r_rate), _ptr(self.r_from), _ptr(self.r_to),
                                  _ptr(self.r_rate), _ptr(src), _ptr(self.eps),
                                  _ptr(self.sink_k), _ptr(self.sink_mask), float(dt),
                                  int(nsteps), _ptr(c), None)
        if rc != 0:
            raise MemoryError("oracle: allocation failed")
        return c

    def balance(self, c, s):
        """(mass, inflow[6], robin_uptake, reaction_total) of species s."""
        lib = _load()
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(
            self.S, self.nz, self.ny, self.nx))
        mass, robin, react = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        inflow = np.zeros(6)
        lib.orc_balance_ext(self.nx, self.ny, self.nz, self.dx, _ptr(self.image), self.S,
                            _ptr(self.D), _ptr(self.robin), _ptr(self.dir_face), len(self.r_rate),
                            _ptr(self.r_from), _ptr(self.r_to), _ptr(self.r_rate), _ptr(self.eps),
                            _ptr(self.sink_k), _ptr(self.sink_mask), _ptr(c), int(s),
                            ctypes.byref(mass), _ptr(inflow), ctypes.byref(robin),
                            ctypes.byref(react))
        return mass.value, inflow, robin.value, react.value

    def plane_flux(self, u, D, axis, i0):
        lib = _load()
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.nz, self.ny, self.nx))
        if self.eps is not None:
            return lib.orc_plane_flux_eps(self.nx, self.ny, self.nz, self.dx, _ptr(self.image),
                                          float(D), _ptr(self.eps), _ptr(u), int(axis), int(i0))
        return lib.orc_plane_flux(self.nx, self.ny, self.nz, self.dx, _ptr(self.image), float(D),
                                  _ptr(u), int(axis), int(i0))


def smooth_diffusivity(phi, d_min, d_max, gamma1, gamma2):
    """D(phi) = d_min + d_max / (1 + exp(-(gamma1 + gamma2 phi))), FP64 (section "Level-set
    method for image-based geometry reconstruction", eq. inhomog_diffusion_coefficient)."""
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64))
    out = np.empty_like(phi)
    _load().orc_smooth_diffusivity(phi.size, _ptr(phi), float(d_min), float(d_max),
                                   float(gamma1), float(gamma2), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# steady state and tortuosity
# ---------------------------------------------------------------------------

def steady_problem(image, axis, D=1.0, dx=1.0):
    """Unit drop along `axis` (0=x,1=y,2=z): Dirichlet 1 on the low face plane and
    0 on the high face plane, no-flux elsewhere."""
    lo, hi = 2 * axis, 2 * axis + 1
    return Problem(image, [D], dx=dx, dirichlet={(0, lo): 1.0, (0, hi): 0.0})


def steady_state(image, axis, solver="cg", tol=1e-12, max_iters=10 ** 7, D=1.0, dx=1.0,
                 initial=None, check_every=50):
    """FP64 steady state of the unit-drop problem.  Returns (u, iters, rel_residual).
    Initial guess on free voxels: ``initial`` if given, else 0."""
    prob = steady_problem(image, axis, D, dx)
    u = prob.initial(0.0)[0]
    if initial is not None:
        f = prob.free_mask(0)
        u[f] = np.asarray(initial, dtype=np.float64).reshape(u.shape)[f]
    u = np.ascontiguousarray(u)
    free_ = np.ascontiguousarray(prob.free_mask(0).astype(np.uint8))
    it, rel = ctypes.c_int64(), ctypes.c_double()
    lib = _load()
    if solver == "cg":
        lib.orc_steady_cg(prob.nx, prob.ny, prob.nz, _ptr(prob.image), _ptr(free_), _ptr(u),
                          float(tol), int(max_iters), ctypes.byref(it), ctypes.byref(rel))
    elif solver == "jacobi":
        lib.orc_steady_jacobi(prob.nx, prob.ny, prob.nz, _ptr(prob.image), _ptr(free_), _ptr(u),
                              float(tol), int(max_iters), int(check_every), ctypes.byref(it),
                              ctypes.byref(rel))
    else:
        raise ValueError(solver)
    return u, it.value, rel.value


def tortuosity_from_field(image, axis, u, D=1.0, dx=1.0):
    """tau = psi * D * dT * A / (Q * L) with Q the diffusive flux out of the inlet
    plane, A the box cross-section, L the distance between the two Dirichlet planes
    and psi the active volume fraction (eq. tortuosity, tau = D_f / D_eff, with the
    effective diffusivity taken from the steady flux).  Returns (tau, Q_in, Q_out)."""
    prob = steady_problem(image, axis, D, dx)
    mass, inflow, _, _ = prob.balance(u[None], 0)
    q_in = inflow[2 * axis]
    q_out = -inflow[2 * axis + 1]
    shape = image.shape[::-1]  # (nx, ny, nz)
    n_ax = shape[axis]
    area = 1.0
    for a in range(3):
        if a != axis:
            area *= shape[a] * dx
    length = (n_ax - 1) * dx
    psi = float(np.count_nonzero(image)) / image.size
    tau = math.inf if q_in <= 0 else psi * D * 1.0 * area / (q_in * length)
    return tau, q_in, q_out


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def adjoint_decay(image, D, k, dt, nsteps, c0, target, dir_faces=(0,), stride=50, dx=1.0):
    """Discrete adjoint of diffusion-decay FTCS.  c0 holds the Dirichlet values.
    Returns (loss, dL/dD, dL/dk, c^N)."""
    lib = _load()
    image = np.ascontiguousarray(image, dtype=np.uint8)
    nz, ny, nx = image.shape
    df = np.zeros(6, dtype=np.uint8)
    for f in dir_faces:
        df[f] = 1
    c0 = np.ascontiguousarray(np.asarray(c0, dtype=np.float64).reshape(nz, ny, nx))
    tg = np.ascontiguousarray(np.asarray(target, dtype=np.float64).reshape(nz, ny, nx))
    cN = np.zeros_like(c0)
    L, gD, gk = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib.orc_adjoint_decay(nx, ny, nz, float(dx), _ptr(image), _ptr(df), float(D), float(k),
                               float(dt), int(nsteps), int(stride), _ptr(c0), _ptr(tg),
                               ctypes.byref(L), ctypes.byref(gD), ctypes.byref(gk), _ptr(cN))
    if rc != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return L.value, gD.value, gk.value, cN


# ---------------------------------------------------------------------------
# active-block index: an independent NumPy scan
# ---------------------------------------------------------------------------

def active_index(image, B):
    """Active-block index of a voxel image (paper: a chunk of B^3 points is stored
    iff it holds at least one inserted point, section "Parallel implementation").

    Returns (block_id int64[nb], nbr int32[nb,6], masks uint64[nb, B^3/64]):
      block_id  linear block id l = (bz*NBy + by)*NBx + bx, ascending
      nbr       index in the list of the face-neighbour block in the order
                -x,+x,-y,+y,-z,+z, or -1 (outside the box or inactive)
      masks     active bits; slot (lz*B + ly)*B + lx is bit (slot % 64) of word slot // 64
    """
    img = np.asarray(image) != 0
    nz, ny, nx = img.shape
    NBz, NBy, NBx = (-(-nz // B)), (-(-ny // B)), (-(-nx // B))
    pad = np.zeros((NBz * B, NBy * B, NBx * B), dtype=bool)
    pad[:nz, :ny, :nx] = img
    blocks = pad.reshape(NBz, B, NBy, B, NBx, B).transpose(0, 2, 4, 1, 3, 5)
    occ = blocks.reshape(NBz, NBy, NBx, B ** 3).any(axis=3)
    block_id = np.flatnonzero(occ.ravel()).astype(np.int64)
    rank = np.full(occ.size, -1, dtype=np.int64)
    rank[block_id] = np.arange(block_id.size)
    bz, rem = np.divmod(block_id, NBy * NBx)
    by, bx = np.divmod(rem, NBx)
    nbr = np.full((block_id.size, 6), -1, dtype=np.int32)
    for f, (dx_, dy_, dz_) in enumerate([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                         (0, 0, -1), (0, 0, 1)]):
        x2, y2, z2 = bx + dx_, by + dy_, bz + dz_
        ok = (x2 >= 0) & (x2 < NBx) & (y2 >= 0) & (y2 < NBy) & (z2 >= 0) & (z2 < NBz)
        lin = (z2 * NBy + y2) * NBx + x2
        r = np.where(ok, rank[np.where(ok, lin, 0)], -1)
        nbr[:, f] = r.astype(np.int32)
    bits = blocks.reshape(NBz * NBy * NBx, B ** 3)[block_id]
    words = max(1, B ** 3 // 64)
    masks = np.zeros((block_id.size, words), dtype=np.uint64)
    for w in range(words):
        chunk = bits[:, w * 64:(w + 1) * 64].astype(np.uint64)
        weights = (np.uint64(1) << np.arange(chunk.shape[1], dtype=np.uint64))
        masks[:, w] = (chunk * weights).sum(axis=1, dtype=np.uint64)
    return block_id, nbr, masks


# ---------------------------------------------------------------------------
# simulated FRAP and the effective diffusion coefficient (section "Calculation of
# effective diffusion coefficient and tortuosity")
# ---------------------------------------------------------------------------

def region_mass(image, c, region, dx=1.0):
    """Sum of c dx^3 over the active voxels with x0 <= x < x1, y0 <= y < y1, z0 <= z < z1
    (region = (x0, x1, y0, y1, z0, z1); arrays are (nz, ny, nx))."""
    x0, x1, y0, y1, z0, z1 = region
    act = np.asarray(image)[z0:z1, y0:y1, x0:x1] != 0
    sub = np.asarray(c, dtype=np.float64)[z0:z1, y0:y1, x0:x1]
    return float(np.sum(sub[act])) * dx ** 3


def frap_curve(prob, c0, region, dt, steps_per_sample, n_samples, species=0):
    """Region mass of one species after k * steps_per_sample FTCS steps, k = 0..n_samples."""
    c = np.array(c0, dtype=np.float64, copy=True)
    out = [region_mass(prob.image, c[species], region, prob.dx)]
    for _ in range(n_samples):
        c = prob.run(c, dt, steps_per_sample)
        out.append(region_mass(prob.image, c[species], region, prob.dx))
    return np.array(out)


def frap_fit(t, f, ds, g, D_ref):
    """D minimising sum_i (f_i - g(t_i D / D_ref))^2, g sampled at j * ds for coefficient
    D_ref (free diffusion depends on D t only; linear interpolation), searched over
    [1e-4, 1] * D_ref s_max / t_max: dense log grid, then a bounded scalar minimiser."""
    from scipy.optimize import minimize_scalar

    t = np.asarray(t, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    s = np.arange(len(g)) * ds
    hi = s[-1] / t.max()

    def err(logsc):
        return float(np.sum((f - np.interp(t * math.exp(logsc), s, g)) ** 2))

    grid = np.linspace(math.log(hi * 1e-4), math.log(hi), 2001)
    e = np.array([err(x) for x in grid])
    k = int(np.argmin(e))
    lo_b, hi_b = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    r = minimize_scalar(err, bounds=(lo_b, hi_b), method="bounded",
                        options={"xatol": 1e-12})
    return math.exp(r.x) * D_ref


def frap_free_space(t, D, half_widths):
    """Mass in the bleached box [-a, a]^3 of free diffusion in all of R^3 from
    c = 1 - indicator(box): the solution factorises over axes,
    c = 1 - prod_d h_d, h = (erf((a - x)/s) + erf((a + x)/s)) / 2, s = sqrt(4 D t), and
    the integral of h over [-a, a] is 2a erf(2a/s) + s (exp(-4a^2/s^2) - 1)/sqrt(pi)."""
    from scipy.special import erf

    t = np.asarray(t, dtype=np.float64)
    vol = 1.0
    prod = np.ones_like(t)
    for a in half_widths:
        vol *= 2 * a
        s = np.sqrt(4 * D * np.maximum(t, 1e-300))
        ia = 2 * a * erf(2 * a / s) + s * (np.exp(-4 * a * a / (s * s)) - 1) / math.sqrt(math.pi)
        prod = prod * np.where(t > 0, ia, 2 * a)
    return vol - prod


# ---------------------------------------------------------------------------
# signed distance of a voxel image (section "Level-set method for image-based geometry
# reconstruction", eq. SDF)
# ---------------------------------------------------------------------------

def signed_distance(image, dx=1.0):
    """phi = (distance from an active voxel centre to the nearest inactive one - 1/2) dx,
    and -(distance to the nearest active one - 1/2) dx at inactive voxels; +-(box
    diagonal) dx if the other phase is empty.  FP64, rounded to FP32 once.  The
    distances come from SciPy's exact Euclidean distance transform."""
    from scipy import ndimage

    img = np.asarray(image) != 0
    diag = math.sqrt(float(np.sum(np.square(img.shape))))
    out = np.empty(img.shape, dtype=np.float64)
    if img.any():
        d_in = ndimage.distance_transform_edt(img) - 0.5 if (~img).any() else np.full(img.shape, diag)
        out[img] = d_in[img] * dx
    if (~img).any():
        d_out = ndimage.distance_transform_edt(~img) - 0.5 if img.any() else np.full(img.shape, diag)
        out[~img] = -d_out[~img] * dx
    return out.astype(np.float32)


# ---------------------------------------------------------------------------
# discrete adjoint with a per-voxel diffusivity factor
# ---------------------------------------------------------------------------

def _neighbours(active):
    """For each direction (-x,+x,-y,+y,-z,+z): (in-box-and-active mask, index shift)."""
    nz, ny, nx = active.shape
    out = []
    for axis, sgn in ((2, -1), (2, 1), (1, -1), (1, 1), (0, -1), (0, 1)):
        m = np.zeros(active.shape, dtype=bool)
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        n = active.shape[axis]
        if sgn < 0:
            dst[axis], src[axis] = slice(1, n), slice(0, n - 1)
        else:
            dst[axis], src[axis] = slice(0, n - 1), slice(1, n)
        m[tuple(dst)] = active[tuple(src)]
        out.append((m & active, tuple(dst), tuple(src)))
    return out


def _shift(u, dst, src):
    v = np.zeros_like(u)
    v[dst] = u[src]
    return v


def adjoint_factor(image, D, k, eps, dt, nsteps, c0, target, dir_faces=(0,), dx=1.0):
    """Discrete adjoint of single-species FTCS with a diffusivity factor e and decay:
        c'_p = c_p + a sum_{q active nb} w_pq (c_q - c_p) - b c_p   (free p),
        a = D dt / dx^2, b = k dt, w_pq = (e_p + e_q) / 2;
    Dirichlet voxels keep c0.  L = 1/2 sum_free (c^N - c*)^2.  With lambda zero off the
    free voxels, lambda^n = the same operator applied to lambda^{n+1}; the gradients are
        dL/dD   = sum_n <lambda^{n+1}, dt/dx^2 sum_q w (c_q - c_p)>,
        dL/dk   = sum_n <lambda^{n+1}, -dt c>,
        dL/de_p = sum_n a/2 sum_{q active nb of p} (c_q - c_p)(lambda_p - lambda_q).
    Returns (loss, dL/dD, dL/dk, dL/de, c^N).  All states are kept (small volumes)."""
    act = np.asarray(image) != 0
    e = np.asarray(eps, dtype=np.float64).reshape(act.shape)
    dirm = np.zeros(act.shape, dtype=bool)
    for f in dir_faces:
        sl = [slice(None)] * 3
        axis = 2 - f // 2
        sl[axis] = 0 if f % 2 == 0 else act.shape[axis] - 1
        dirm[tuple(sl)] = True
    dirm &= act
    free = act & ~dirm
    nb = _neighbours(act)
    a, b = D * dt / dx ** 2, k * dt
    w = [0.5 * (e + _shift(e, dst, src)) * m for (m, dst, src) in nb]

    def lap(u):
        return sum(wd * (_shift(u, dst, src) - u) for wd, (m, dst, src) in zip(w, nb))

    c = np.where(act, np.asarray(c0, dtype=np.float64).reshape(act.shape), 0.0)
    states = [c]
    for _ in range(nsteps):
        c = np.where(free, c + a * lap(c) - b * c, c)
        states.append(c)
    tg = np.asarray(target, dtype=np.float64).reshape(act.shape)
    r = np.where(free, c - tg, 0.0)
    loss = 0.5 * float(np.sum(r * r))
    lam = r
    gD = gk = 0.0
    ge = np.zeros(act.shape)
    for n in range(nsteps - 1, -1, -1):
        cn = states[n]
        gD += float(np.sum(lam * lap(cn))) * dt / dx ** 2
        gk += float(np.sum(lam * cn)) * -dt
        for (m, dst, src) in nb:
            ge += np.where(m, 0.5 * a * (_shift(cn, dst, src) - cn) * (lam - _shift(lam, dst, src)), 0.0)
        lam = np.where(free, lam + a * lap(lam) - b * lam, 0.0)
    return loss, gD, gk, np.where(act, ge, 0.0), states[-1]
