"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test fixes a value the mathematics (or the paper) determines, so that a
dropped term, a wrong sign or a swapped index in the oracle fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------------------
# diffusion + mirror rule + Dirichlet: exact discrete closed form (1-D slab)
# ---------------------------------------------------------------------------

def slab_closed_form(N, s, n):
    """FTCS on i = 0..N-1 with u_0 = 1 held, u = 0 initially, zero flux past i = N-1.
    Eigenvectors sin(theta_m i), theta_m = (2m+1) pi / (2N-1), m = 0..N-2;
    eigenvalues mu_m = 1 - 4 s sin^2(theta_m / 2)."""
    i = np.arange(N, dtype=np.float64)
    u = np.ones(N)
    for m in range(N - 1):
        th = (2 * m + 1) * math.pi / (2 * N - 1)
        a = -np.sin(th * i[1:]).sum() / ((2 * N - 1) / 4.0)
        u += a * (1 - 4 * s * math.sin(th / 2) ** 2) ** n * np.sin(th * i)
    return u


@pytest.mark.parametrize("N,D,dt,n", [(20, 1.0, 0.1, 50), (33, 0.4, 0.25, 400), (9, 1.0, 0.15, 1000)])
def test_slab_discrete_closed_form(oracle_mod, N, D, dt, n):
    img = W.slab_box(N, ny=3, nz=2)
    prob = oracle_mod.Problem(img, [D], dirichlet={(0, 0): 1.0})
    c = prob.run(prob.initial(), dt, n)[0]
    ref = slab_closed_form(N, D * dt, n)
    for k in range(2):
        for j in range(3):
            np.testing.assert_allclose(c[k, j], ref, rtol=0, atol=1e-12)


def test_slab_axis_symmetry(oracle_mod):
    """The same slab along y and along z gives the same profile (no axis is special)."""
    N = 17
    ref = slab_closed_form(N, 0.1, 80)
    for f, shape in [(2, (2, N, 3)), (4, (N, 3, 2))]:
        prob = oracle_mod.Problem(np.ones(shape, np.uint8), [1.0], dirichlet={(0, f): 1.0})
        c = prob.run(prob.initial(), 0.1, 80)[0]
        prof = c[0, :, 0] if f == 2 else c[:, 0, 0]
        np.testing.assert_allclose(prof, ref, atol=1e-12)


def test_slab_high_face_dirichlet(oracle_mod):
    """Dirichlet on the +x face gives the mirrored profile."""
    N = 15
    prob = oracle_mod.Problem(W.slab_box(N, 2, 2), [1.0], dirichlet={(0, 1): 1.0})
    c = prob.run(prob.initial(), 0.1, 60)[0]
    np.testing.assert_allclose(c[0, 0, ::-1], slab_closed_form(N, 0.1, 60), atol=1e-12)


# ---------------------------------------------------------------------------
# continuum: erfc before the front reaches the far wall, order 2 in dx
# ---------------------------------------------------------------------------

def test_erfc_convergence_order_two(oracle_mod):
    from scipy.special import erfc

    t_end, D, Lx = 0.01, 1.0, 1.0
    errs = []
    for N in (41, 81, 161):
        dx = Lx / (N - 1)
        dt = 0.1 * dx * dx / D
        n = int(round(t_end / dt))
        prob = oracle_mod.Problem(W.slab_box(N, 1, 1), [D], dx=dx, dirichlet={(0, 0): 1.0})
        c = prob.run(prob.initial(), dt, n)[0, 0, 0]
        x = np.arange(N) * dx
        exact = erfc(x / (2 * math.sqrt(D * n * dt)))
        errs.append(np.abs(c - exact).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < o < 2.3 for o in orders), (errs, orders)


# ---------------------------------------------------------------------------
# curved no-flux walls: the paper's manufactured solution in a disk
# ---------------------------------------------------------------------------

def _mms_error(oracle_mod, k):
    g = GOLD["mms_disk"]
    Bc, D = g["B"], g["D"]
    n = g["smallest_grid_nodes"] * 2 ** k
    rc = (g["nodes_across_diameter_at_smallest_grid"] // 2) * 2 ** k
    img, _, r, h = W.disk_cylinder(n, rc)
    dt = g["dt_over_h2"] * h * h
    nsteps = int(round(g["t_final"] / dt))
    prob = oracle_mod.Problem(img, [D], dx=h)
    U = lambda t: (r ** 3 / 3 - r ** 4 / 4) * math.exp(-Bc * t)
    f = lambda t: (Bc / 4 * r ** 4 - Bc / 3 * r ** 3 + 4 * r ** 2 - 3 * r) * math.exp(-Bc * t)
    c = prob.apply_dirichlet(U(0.0)[None])
    act = img != 0
    for step in range(nsteps):
        src = np.where(act, f(step * dt), 0.0)
        c = prob.run(c, dt, 1, source=src[None])
    e = (c[0] - U(nsteps * dt))[act]
    return math.sqrt(np.mean(e ** 2)), np.abs(e).max()


def test_mms_disk_convergence(oracle_mod):
    """Paper's verification case: diffusion in the unit disk with no-flux walls
    imposed by the mirror rule; the observed order lies between 1 and 2."""
    errs = [_mms_error(oracle_mod, k) for k in range(4)]
    l2 = [e[0] for e in errs]
    orders = [math.log2(l2[i] / l2[i + 1]) for i in range(3)]
    lo, hi = GOLD["mms_disk"]["expected_order_range"]
    assert all(l2[i + 1] < l2[i] for i in range(3)), l2
    mean_order = float(np.mean(orders))
    assert lo - 0.1 < mean_order < hi + 0.3, (l2, orders)


# ---------------------------------------------------------------------------
# conservation and balance
# ---------------------------------------------------------------------------

def _porous(n=20, seed=7):
    img, _ = W.boolean_spheres(n, 0.5, 2.0, 4.0, seed=seed)
    return img


def test_mass_conserved_no_flux(oracle_mod):
    img = _porous(24)
    prob = oracle_mod.Problem(img, [1.0])
    rng = np.random.default_rng(11)
    c = prob.apply_dirichlet(rng.uniform(0, 1, (1,) + img.shape))
    m0 = prob.balance(c, 0)[0]
    c2 = prob.run(c, 0.15, 300)
    m1 = prob.balance(c2, 0)[0]
    assert abs(m1 - m0) / m0 < 1e-13
    # the field moved (so the test is not vacuous)
    assert np.abs(c2 - c).max() > 1e-2


def test_discrete_balance_each_step(oracle_mod):
    """M' - M = dt * (sum inflow - robin uptake + reactions), per species."""
    img = _porous(18, seed=3)
    img[:, :, 0] = 1  # make the Dirichlet plane connect
    prob = oracle_mod.Problem(img, [1.0, 0.4], dx=0.7, robin={1: 0.05},
                              dirichlet={(0, 0): 1.0}, reactions=[(0, 1, 0.01)])
    dt = 0.1 * 0.49
    rng = np.random.default_rng(5)
    c = prob.apply_dirichlet(rng.uniform(0, 1, (2,) + img.shape))
    for _ in range(5):
        c2 = prob.run(c, dt, 1)
        for s in range(2):
            m0, infl, rb, re = prob.balance(c, s)
            m1 = prob.balance(c2, s)[0]
            pred = dt * (infl.sum() - rb + re)
            assert abs((m1 - m0) - pred) <= 1e-12 * max(1.0, abs(m0)), (s, m1 - m0, pred)
        c = c2
    # both balance terms were non-trivial
    assert prob.balance(c, 0)[1][0] > 0 and prob.balance(c, 1)[2] > 0


def test_a_plus_b_conserved(oracle_mod):
    img = _porous(16, seed=9)
    prob = oracle_mod.Problem(img, [1.0, 0.4], reactions=[(0, 1, 0.05)])
    rng = np.random.default_rng(2)
    c = prob.apply_dirichlet(rng.uniform(0, 1, (2,) + img.shape))
    a0, b0 = prob.balance(c, 0)[0], prob.balance(c, 1)[0]
    c = prob.run(c, 0.1, 200)
    a1, b1 = prob.balance(c, 0)[0], prob.balance(c, 1)[0]
    assert abs((a1 + b1) - (a0 + b0)) / (a0 + b0) < 1e-13
    # A converted into B at the first-order rate: A(t) = A0 (1 - k dt)^n (uniform in space)
    assert a1 == pytest.approx(a0 * (1 - 0.05 * 0.1) ** 200, rel=1e-12)
    assert b1 > b0


def test_uniform_decay_closed_form(oracle_mod):
    img = _porous(16, seed=4)
    k, dt, n = 0.02, 0.1, 500
    prob = oracle_mod.Problem(img, [0.8], reactions=[(0, -1, k)])
    c = prob.run(prob.initial(0.7), dt, n)[0]
    np.testing.assert_allclose(c[img != 0], 0.7 * (1 - k * dt) ** n, rtol=1e-13)
    assert np.all(c[img == 0] == 0)


@pytest.mark.parametrize("pos,nwall", [((5, 5, 5), 6), ((0, 5, 5), 5), ((0, 0, 0), 3), ((10, 0, 5), 4), ((3, 10, 0), 4)])
def test_isolated_voxel_robin(oracle_mod, pos, nwall):
    """An isolated active voxel loses c * k_R * n_wall * dx^2 per unit time; box faces
    are not walls."""
    img = np.zeros((11, 11, 11), np.uint8)
    x, y, z = pos
    img[z, y, x] = 1
    kR, dt, dx, n = 0.05, 0.1, 1.0, 300
    prob = oracle_mod.Problem(img, [1.0], robin={0: kR})
    c = prob.run(prob.initial(1.0), dt, n)[0]
    assert c[z, y, x] == pytest.approx((1 - dt * kR * nwall / dx) ** n, rel=1e-13)


def test_robin_zero_is_no_flux(oracle_mod):
    img = _porous(14, seed=1)
    rng = np.random.default_rng(0)
    p0 = oracle_mod.Problem(img, [1.0])
    p1 = oracle_mod.Problem(img, [1.0], robin={0: 0.0})
    c = p0.apply_dirichlet(rng.uniform(0, 1, (1,) + img.shape))
    np.testing.assert_array_equal(p0.run(c, 0.1, 20), p1.run(c, 0.1, 20))


def test_brute_force_single_voxel_updates(oracle_mod):
    """One step at a handful of voxels against the update written out by hand."""
    img = _porous(10, seed=12)
    rng = np.random.default_rng(8)
    prob = oracle_mod.Problem(img, [0.9, 0.3], dx=1.3, robin={0: 0.02, 1: 0.07},
                              dirichlet={(1, 3): 0.5}, reactions=[(0, 1, 0.03), (1, -1, 0.01)])
    c = prob.apply_dirichlet(rng.uniform(0, 1, (2,) + img.shape))
    dt = 0.05
    c1 = prob.run(c, dt, 1)
    nz, ny, nx = img.shape
    act = img != 0
    free1 = prob.free_mask(1)
    checked = 0
    for (z, y, x) in np.argwhere(act)[:: 37]:
        for s in range(2):
            if s == 1 and not free1[z, y, x]:
                assert c1[s, z, y, x] == c[s, z, y, x]
                continue
            lap, nw = 0.0, 0
            for dz, dy, dxx in [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]:
                zz, yy, xx = z + dz, y + dy, x + dxx
                if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
                    continue
                if act[zz, yy, xx]:
                    lap += c[s, zz, yy, xx] - c[s, z, y, x]
                else:
                    nw += 1
            D = prob.D[s]
            v = c[s, z, y, x] + dt * D * lap / 1.3 ** 2 - dt * prob.robin[s] * nw * c[s, z, y, x] / 1.3
            if s == 0:
                v -= dt * 0.03 * c[0, z, y, x]
            else:
                v += dt * 0.03 * c[0, z, y, x] - dt * 0.01 * c[1, z, y, x]
            assert c1[s, z, y, x] == pytest.approx(v, rel=1e-13, abs=1e-15)
            checked += 1
    assert checked > 20


# ---------------------------------------------------------------------------
# steady state and tortuosity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tortuosity_straight_channels(oracle_mod, axis):
    img = W.straight_channels(16, 12, 12, period=4, width=2)
    if axis == 1:
        img = np.ascontiguousarray(img.transpose(0, 2, 1))
    elif axis == 2:
        img = np.ascontiguousarray(img.transpose(2, 1, 0))
    u, it, rel = oracle_mod.steady_state(img, axis, "cg", tol=1e-13)
    assert rel < 1e-12
    tau, qin, qout = oracle_mod.tortuosity_from_field(img, axis, u)
    assert tau == pytest.approx(1.0, rel=1e-10)
    assert qin == pytest.approx(qout, rel=1e-10)


def test_tortuosity_all_pore_and_linear_profile(oracle_mod):
    img = W.slab_box(10, 6, 5)
    u, _, _ = oracle_mod.steady_state(img, 0, "cg", tol=1e-14)
    np.testing.assert_allclose(u[0, 0], 1 - np.arange(10) / 9.0, atol=1e-12)
    tau, _, _ = oracle_mod.tortuosity_from_field(img, 0, u)
    assert tau == pytest.approx(1.0, rel=1e-12)


def test_tortuosity_non_percolating_is_infinite(oracle_mod):
    img = W.slab_box(12, 6, 6)
    img[:, :, 5] = 0  # a solid wall across x
    u, _, _ = oracle_mod.steady_state(img, 0, "cg", tol=1e-13)
    tau, qin, _ = oracle_mod.tortuosity_from_field(img, 0, u)
    assert math.isinf(tau) and abs(qin) < 1e-12


def test_jacobi_and_cg_agree_and_flux_is_constant(oracle_mod):
    img = _porous(16, seed=21)
    img[:, :, 0] = 1
    img[:, :, -1] = 1
    u1, it1, r1 = oracle_mod.steady_state(img, 0, "cg", tol=1e-13)
    u2, it2, r2 = oracle_mod.steady_state(img, 0, "jacobi", tol=1e-12, max_iters=2_000_000)
    assert r1 < 1e-13 and r2 < 1e-12
    np.testing.assert_allclose(u1, u2, atol=1e-9)
    tau, qin, qout = oracle_mod.tortuosity_from_field(img, 0, u1)
    assert 1.0 < tau < 10.0
    prob = oracle_mod.steady_problem(img, 0)
    for i in range(0, 15):
        assert prob.plane_flux(u1, 1.0, 0, i) == pytest.approx(qin, rel=1e-9)
    assert qout == pytest.approx(qin, rel=1e-9)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def _adj_case(oracle_mod, n=12, seed=3):
    img, _ = W.boolean_spheres(n, 0.5, 2.0, 3.5, seed=seed)
    img[:, :, 0] = 1
    prob_t = oracle_mod.Problem(img, [1.0], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, 0.01)])
    c0 = prob_t.initial()
    target = prob_t.run(c0, 0.1, 120)[0]
    return img, c0[0], target


def test_adjoint_matches_central_fd(oracle_mod):
    img, c0, target = _adj_case(oracle_mod)
    D, k, dt, n = 0.8, 0.02, 0.1, 120
    L, gD, gk, _ = oracle_mod.adjoint_decay(img, D, k, dt, n, c0, target, stride=7)
    h = 1e-4

    def loss(Dv, kv):
        return oracle_mod.adjoint_decay(img, Dv, kv, dt, n, c0, target, stride=50)[0]

    fdD = (loss(D + h, k) - loss(D - h, k)) / (2 * h)
    fdk = (loss(D, k + h) - loss(D, k - h)) / (2 * h)
    assert gD == pytest.approx(fdD, rel=1e-6)
    assert gk == pytest.approx(fdk, rel=1e-6)
    assert abs(gD) > 1e-3 and abs(gk) > 1e-3


def test_adjoint_stride_independent(oracle_mod):
    img, c0, target = _adj_case(oracle_mod, n=10, seed=5)
    r = [oracle_mod.adjoint_decay(img, 0.8, 0.02, 0.1, 75, c0, target, stride=s)[:3]
         for s in (1, 10, 50, 100)]
    for x in r[1:]:
        np.testing.assert_allclose(x, r[0], rtol=1e-13)


def test_adjoint_uniform_closed_form(oracle_mod):
    """Uniform field, no flux, no Dirichlet: dL/dD = 0 exactly and
    dL/dk = -n_free * (c^N - c*) * c0 * N dt (1 - k dt)^(N-1)."""
    img = _porous(10, seed=2)
    c0v, k, dt, N = 0.6, 0.02, 0.1, 40
    c0 = np.where(img != 0, c0v, 0.0)
    target = np.where(img != 0, 0.3, 0.0)
    L, gD, gk, cN = oracle_mod.adjoint_decay(img, 0.8, k, dt, N, c0, target, dir_faces=())
    n_free = int(img.sum())
    cNv = c0v * (1 - k * dt) ** N
    assert gD == 0.0
    assert gk == pytest.approx(-n_free * (cNv - 0.3) * c0v * N * dt * (1 - k * dt) ** (N - 1),
                               rel=1e-12)
    assert L == pytest.approx(0.5 * n_free * (cNv - 0.3) ** 2, rel=1e-12)


# ---------------------------------------------------------------------------
# active-block index: NumPy scan vs brute force, and lattice counts
# ---------------------------------------------------------------------------

def _index_brute(img, B):
    nz, ny, nx = img.shape
    NB = [-(-nx // B), -(-ny // B), -(-nz // B)]
    occ = set()
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if img[z, y, x]:
                    occ.add(((z // B) * NB[1] + y // B) * NB[0] + x // B)
    ids = sorted(occ)
    where = {l: i for i, l in enumerate(ids)}
    nbr = []
    for l in ids:
        bx, by, bz = l % NB[0], (l // NB[0]) % NB[1], l // (NB[0] * NB[1])
        row = []
        for d in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
            x2, y2, z2 = bx + d[0], by + d[1], bz + d[2]
            if 0 <= x2 < NB[0] and 0 <= y2 < NB[1] and 0 <= z2 < NB[2]:
                row.append(where.get((z2 * NB[1] + y2) * NB[0] + x2, -1))
            else:
                row.append(-1)
        nbr.append(row)
    return ids, nbr


@pytest.mark.parametrize("seed,B", [(0, 4), (1, 8), (2, 4), (3, 8), (4, 8)])
def test_index_scan_vs_brute_force(oracle_mod, seed, B):
    img = W.random_tiny_geometry(seed, density=0.02 if seed % 2 else None)
    ids, nbr, masks = oracle_mod.active_index(img, B)
    ids2, nbr2 = _index_brute(img, B)
    assert list(ids) == ids2
    assert nbr.tolist() == nbr2
    # mask bits
    nz, ny, nx = img.shape
    NBx, NBy = -(-nx // B), -(-ny // B)
    for b, l in enumerate(ids):
        bx, by, bz = l % NBx, (l // NBx) % NBy, l // (NBx * NBy)
        for slot in range(B ** 3):
            lx, ly, lz = slot % B, (slot // B) % B, slot // (B * B)
            x, y, z = bx * B + lx, by * B + ly, bz * B + lz
            want = x < nx and y < ny and z < nz and img[z, y, x] != 0
            got = (int(masks[b, slot // 64]) >> (slot % 64)) & 1
            assert got == int(want)


def test_single_sphere_active_count(oracle_mod):
    n, c, r = 24, (11.3, 12.1, 10.7), 7.2
    img, _ = W.single_sphere(n, c, r)
    count = 0
    for z in range(n):
        for y in range(n):
            for x in range(n):
                count += (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 > r * r
    _, _, masks = oracle_mod.active_index(img, 8)
    bits = sum(bin(int(w)).count("1") for w in masks.ravel())
    assert bits == count == int(img.sum())


# ---------------------------------------------------------------------------
# input generators (not the method, but pinned as well)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_edt_sdf_equals_brute_force(seed):
    img = W.random_tiny_geometry(seed, shape=(7, 9, 8))
    if img.all() or not img.any():
        img[0, 0, 0] ^= 1
    np.testing.assert_allclose(W.sdf_from_image(img), W.sdf_brute_force(img), atol=1e-6)


def test_sphere_sdf_edt_first_order():
    img, phi = W.single_sphere(32, (15.5, 16.2, 15.8), 9.3)
    sdf = W.sdf_from_image(img)
    assert np.all(np.sign(sdf) == np.where(img != 0, 1, -1))
    assert np.abs(sdf - phi).max() <= 1.0


def test_sphere_packing_exact_sdf():
    img, sdf, cen, rad = W.disjoint_sphere_packing(64, 40, 4.0, 8.0, seed=1)
    assert len(rad) == 40 and img.shape == (64, 64, 64)
    assert np.all((sdf > 0) == (img != 0))
    # realised porosity of 40 disjoint spheres r~U(4,8) in 64^3 is ~0.85
    assert 0.80 < img.mean() < 0.92
    for i in range(40):
        for j in range(i):
            assert np.linalg.norm(cen[i] - cen[j]) >= rad[i] + rad[j]
