"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random geometries and states workload parameters.  It holds
none of the reaction-diffusion arithmetic: no stencil, no reduction, no solver.

The paper simulates in segmented micro-CT volumes (a CaCO3 packed bed and a
reticulate porous ceramic, section "Application example 1/2"); those volumes are
not public, so the seeded volumes below stand in for them.  Every generator takes
an explicit seed and uses ``numpy.random.default_rng(seed)`` (PCG64).

Conventions (shared with the C-ABI): arrays are C-ordered ``(nz, ny, nx)`` with x
fastest; voxel (i, j, k) has its centre at (i, j, k) * dx; ``image`` is uint8 with
1 = inside the diffusion domain Omega (level set phi > 0, section "Level-set
method", eq. SDF) and 0 = outside.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "disjoint_sphere_packing",
    "boolean_spheres",
    "gaussian_random_field_volume",
    "sdf_from_image",
    "sdf_brute_force",
    "slab_box",
    "straight_channels",
    "single_sphere",
    "disk_cylinder",
    "Workload",
    "workload",
    "random_tiny_geometry",
]


# ---------------------------------------------------------------------------
# geometries
# ---------------------------------------------------------------------------

def _grid_coords(n_zyx):
    nz, ny, nx = n_zyx
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return z, y, x


def disjoint_sphere_packing(n=64, n_spheres=40, rmin=4.0, rmax=8.0, seed=1, max_tries=200000):
    """Random sequential addition of ``n_spheres`` non-overlapping solid balls.

    Radii r ~ U(rmin, rmax) (continuous), centres uniform in [r, n-1-r]^3, a
    candidate is rejected if it overlaps an accepted ball.  The pore space (the
    diffusion domain) is the complement of the union.  For disjoint balls the
    exact signed distance to the pore/solid interface is
    ``phi(x) = min_i (|x - c_i| - r_i)`` (positive in the pore).

    Returns (image u8 (n,n,n), sdf f32 (n,n,n), centres (k,3) as (x,y,z), radii).
    """
    rng = np.random.default_rng(seed)
    centres, radii = [], []
    tries = 0
    while len(radii) < n_spheres:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("sphere packing: too many rejections")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r, (n - 1) - r, size=3)
        ok = True
        for c2, r2 in zip(centres, radii):
            if np.linalg.norm(c - c2) < r + r2:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    centres = np.array(centres)
    radii = np.array(radii)
    z, y, x = _grid_coords((n, n, n))
    phi = np.full((n, n, n), np.inf)
    for (cx, cy, cz), r in zip(centres, radii):
        d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - r
        np.minimum(phi, d, out=phi)
    image = (phi > 0).astype(np.uint8)
    return image, phi.astype(np.float32), centres, radii


def boolean_spheres(n, porosity, rmin, rmax, seed, active="pore"):
    """Boolean model: overlapping balls with Poisson centres.

    Centres form a Poisson process of intensity lambda = -ln(p)/E[V] in the box
    extended by ``rmax`` on every side, radii r ~ U(rmin, rmax), E[V] = 4/3 pi E[r^3].
    With ``active="pore"`` the balls are solid and the pore is their complement
    (expected pore fraction p = ``porosity``).  With ``active="solid"`` the balls are
    pores of total fraction ``porosity`` and the returned image marks the solid
    matrix (the phase heat conducts through).

    ``n`` is an int (cube) or a (nz, ny, nx) tuple.  Returns (image u8, info dict).
    """
    if isinstance(n, int):
        shape = (n, n, n)
    else:
        shape = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    er3 = (rmax ** 4 - rmin ** 4) / (4.0 * (rmax - rmin))  # E[r^3] for r ~ U(rmin, rmax)
    ev = 4.0 / 3.0 * math.pi * er3
    # the active phase is always the complement of the balls; its expected volume
    # fraction is exp(-lambda E[V])
    keep = porosity if active == "pore" else 1.0 - porosity
    lam = -math.log(keep) / ev
    ext = np.array([s + 2 * rmax for s in shape[::-1]], dtype=np.float64)  # (x, y, z)
    n_balls = rng.poisson(lam * float(np.prod(ext)))
    cen = rng.uniform(0.0, 1.0, size=(n_balls, 3)) * ext - rmax
    rad = rng.uniform(rmin, rmax, size=n_balls)
    balls = np.zeros(shape, dtype=bool)
    nz, ny, nx = shape
    for (cx, cy, cz), r in zip(cen, rad):
        x0, x1 = max(0, int(math.floor(cx - r))), min(nx - 1, int(math.ceil(cx + r)))
        y0, y1 = max(0, int(math.floor(cy - r))), min(ny - 1, int(math.ceil(cy + r)))
        z0, z1 = max(0, int(math.floor(cz - r))), min(nz - 1, int(math.ceil(cz + r)))
        if x0 > x1 or y0 > y1 or z0 > z1:
            continue
        zz = np.arange(z0, z1 + 1, dtype=np.float64)[:, None, None]
        yy = np.arange(y0, y1 + 1, dtype=np.float64)[None, :, None]
        xx = np.arange(x0, x1 + 1, dtype=np.float64)[None, None, :]
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
        balls[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1] |= inside
    image = (~balls).astype(np.uint8)
    info = {"n_balls": int(n_balls), "intensity": lam, "porosity_target": porosity,
            "active_fraction": float(image.mean())}
    return image, info


def gaussian_random_field_volume(n=512, corr_len=12.0, porosity=0.3, seed=2):
    """Soil-like volume: periodic Gaussian random field thresholded at a quantile.

    White noise is filtered in Fourier space with a Gaussian kernel of standard
    deviation sigma = corr_len / sqrt(2), so the field's covariance is
    exp(-r^2 / (2 corr_len^2)).  The pore (active) phase is the set of voxels below
    the ``porosity`` quantile, i.e. exactly that fraction up to ties.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n), dtype=np.float32)
    spec = np.fft.rfftn(noise)
    del noise
    sigma = corr_len / math.sqrt(2.0)
    # The Gaussian kernel factorises over the axes; each 1-D factor is evaluated with
    # the C library's exp (one value per frequency), and the products are plain IEEE
    # multiplications, so the volume is the same on every host CPU (numpy's vector exp
    # differs between instruction sets in the last bit, which can move a voxel across
    # the threshold).
    def factor(freqs):
        return np.array([math.exp(-0.5 * sigma * sigma * (2 * math.pi * f) ** 2) for f in freqs],
                        dtype=np.float32)

    gz = factor(np.fft.fftfreq(n))
    gy = factor(np.fft.fftfreq(n))[:, None]
    gx = factor(np.fft.rfftfreq(n))[None, :]
    for z in range(n):
        spec[z] *= gz[z] * gy * gx
    field_ = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2)).astype(np.float32)
    del spec
    thr = np.quantile(field_[:: 2, :: 2, :: 2] if n > 256 else field_, porosity)
    image = (field_ < thr).astype(np.uint8)
    return image


def sdf_from_image(image):
    """Signed distance for a binary image via an exact Euclidean distance transform.

    Pore voxels get d_E(p, nearest solid voxel centre) - 1/2; solid voxels get
    -(d_E(p, nearest pore voxel centre) - 1/2).  Only sign(phi) reaches the
    constant-D stepping, and the sign always matches ``image``.
    """
    from scipy import ndimage

    img = image.astype(bool)
    sdf = np.empty(image.shape, dtype=np.float32)
    if img.all():
        sdf[...] = np.float32(np.sqrt(np.sum(np.square(image.shape))))
        return sdf
    if not img.any():
        sdf[...] = -np.float32(np.sqrt(np.sum(np.square(image.shape))))
        return sdf
    d_in = ndimage.distance_transform_edt(img)
    d_out = ndimage.distance_transform_edt(~img)
    sdf[...] = np.where(img, d_in - 0.5, -(d_out - 0.5))
    return sdf


def sdf_brute_force(image):
    """Brute-force version of :func:`sdf_from_image` (O(N^2); tiny volumes only)."""
    img = image.astype(bool)
    pts = np.argwhere(np.ones_like(img)).astype(np.float64)
    pore = np.argwhere(img).astype(np.float64)
    solid = np.argwhere(~img).astype(np.float64)
    out = np.empty(img.size)
    flat = img.ravel()
    for i, p in enumerate(pts):
        other = solid if flat[i] else pore
        if len(other) == 0:
            out[i] = np.inf if flat[i] else -np.inf
            continue
        d = np.sqrt(((other - p) ** 2).sum(axis=1).min())
        out[i] = d - 0.5 if flat[i] else -(d - 0.5)
    return out.reshape(img.shape)


def slab_box(nx, ny=4, nz=4):
    """All-pore box (every voxel active)."""
    return np.ones((nz, ny, nx), dtype=np.uint8)


def straight_channels(nx, ny, nz, period=4, width=2):
    """Square channels running along x: voxel active iff (y mod period < width) and
    (z mod period < width)."""
    z, y, _ = np.indices((nz, ny, 1))
    m = ((y % period) < width) & ((z % period) < width)
    return np.broadcast_to(m, (nz, ny, nx)).astype(np.uint8).copy()


def single_sphere(n, centre, radius, inside_active=False):
    """One ball; exact SDF.  ``inside_active`` selects which side is Omega."""
    z, y, x = _grid_coords((n, n, n))
    cx, cy, cz = centre
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - radius  # >0 outside
    phi = -d if inside_active else d
    return (phi > 0).astype(np.uint8), phi.astype(np.float32)


def disk_cylinder(n, radius_cells):
    """z-invariant unit-disk domain on an n x n grid (nz = 1).

    The disk of radius R = 1 is centred in a square of side ``n*h`` with
    h = 1/radius_cells, grid node (i, j) at ((i + 0.5) - n/2) * h.  Returns
    (image (1,n,n) u8, sdf (1,n,n) f64, r (1,n,n) f64, h).
    """
    h = 1.0 / radius_cells
    c = (np.arange(n, dtype=np.float64) + 0.5 - n / 2.0) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2)
    phi = 1.0 - r
    return (phi > 0).astype(np.uint8)[None], phi[None], r[None], h


def random_tiny_geometry(seed, shape=None, density=None):
    """A random small volume for property tests: random shape in 1..24 per axis,
    random Bernoulli density, plus a few isolated voxels."""
    rng = np.random.default_rng(seed)
    if shape is None:
        shape = tuple(int(v) for v in rng.integers(1, 25, size=3))
    if density is None:
        density = float(rng.uniform(0.05, 0.95))
    img = (rng.random(shape) < density).astype(np.uint8)
    return img


# ---------------------------------------------------------------------------
# the five workloads (parameters + geometry recipe)
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    shape: tuple  # (nz, ny, nx)
    dx: float
    block_edge: int
    species_D: list
    reactions: list = field(default_factory=list)  # (from, to, rate); to = -1: decay
    robin: dict = field(default_factory=dict)  # species -> k_R
    dirichlet: dict = field(default_factory=dict)  # (species, face) -> value
    dt: float = 0.1
    steps: int = 0
    seed: int = 0
    note: str = ""


def workload(name, small=False):
    """Parameters of the named workload.  ``small`` shrinks the volume (same recipe)
    for tests that the oracle must finish in seconds.  Geometry comes from
    :func:`workload_geometry`."""
    if name == "spheres64":
        return Workload("spheres64", (64, 64, 64), 1.0, 8, [1.0],
                        dirichlet={(0, 0): 1.0}, dt=0.1, steps=1000, seed=1,
                        note="40 disjoint solid spheres r~U(4,8); D=1; c=1 on the x=0 face")
    if name == "soil512":
        n = 96 if small else 512
        return Workload("soil512", (n, n, n), 1.0, 8, [1.0, 0.4],
                        reactions=[(0, 1, 0.01)], robin={1: 0.05},
                        dirichlet={(0, 0): 1.0}, dt=0.1, steps=10000, seed=2,
                        note="GRF corr 12 thresholded to porosity 0.3; A->B k=0.01; Robin on B k=0.05")
    if name == "foam1024":
        n = 128 if small else 1024
        return Workload("foam1024", (n, n, n), 1.0, 8, [1.0], dt=0.15, steps=1000, seed=3,
                        note="solid matrix of a ceramic with overlapping pore spheres r~U(10,30), porosity 0.15")
    if name == "decay256":
        n = 64 if small else 256
        return Workload("decay256", (n, n, n), 1.0, 8, [0.8], reactions=[(0, -1, 0.02)],
                        dirichlet={(0, 0): 1.0}, dt=0.1, steps=2000, seed=5,
                        note="boolean sphere packing p=0.5; diffusion-decay; adjoint target D=1,k=0.01")
    raise KeyError(name)


def workload_geometry(name, small=False):
    """(image u8, sdf f32 or None) for a named workload (seeded)."""
    w = workload(name, small)
    n = w.shape[0]
    if name == "spheres64":
        img, sdf, _, _ = disjoint_sphere_packing(64, 40, 4.0, 8.0, seed=w.seed)
        return img, sdf
    if name == "soil512":
        img = gaussian_random_field_volume(n, 12.0, 0.3, seed=w.seed)
        return img, None
    if name == "foam1024":
        img, _ = boolean_spheres(n, 0.15, 10.0, 30.0, seed=w.seed, active="solid")
        return img, None
    if name == "decay256":
        img, _ = boolean_spheres(n, 0.5, 4.0, 8.0, seed=w.seed, active="pore")
        return img, None
    raise KeyError(name)


def batch_geometries(count=64, seed=4, nmin=64, nmax=256, scale=1.0):
    """The batch of sphere packings: geometry i uses seed stream (seed, i), edge
    N ~ U{nmin..nmax} (times ``scale`` for reduced tests), porosity p ~ U(0.3, 0.7),
    boolean solid spheres r ~ U(4, 8).  Returns a list of (image, info)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(nmin, nmax + 1))
        n = max(4, int(round(n * scale)))
        p = float(rng.uniform(0.3, 0.7))
        sub = int(rng.integers(0, 2 ** 31))
        img, info = boolean_spheres(n, p, 4.0, 8.0, seed=sub, active="pore")
        info["n"] = n
        out.append((img, info))
    return out
