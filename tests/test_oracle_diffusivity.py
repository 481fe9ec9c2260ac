"""Pins of the oracle's inhomogeneous diffusion (a per-voxel diffusivity factor e, the
arithmetic mean of D at the two voxels of a face, appendix "Code examples") and of the
smooth diffusivity D(phi) of section "Level-set method for image-based geometry
reconstruction", eq. inhomog_diffusion_coefficient.

What fixes each value:
  * a constant factor e is the same as scaling D by e (reduces to the pinned
    homogeneous step);
  * a closed box conserves mass for any e (the face fluxes are antisymmetric only
    when both sides use the same face coefficient);
  * a 1-D chain with Dirichlet ends is a series of conductances: its exact discrete
    steady state (Kirchhoff) is a fixed point of the step, and the balance reports the
    one through-flux on both faces;
  * D(x) = 1 + x / L between c = 1 and c = 0 has the continuum steady state
    1 - ln(1 + x / L) / ln 2, approached at second order;
  * D(phi) against scipy's logistic function, its limits and its point symmetry.
"""
import math

import numpy as np
import pytest
from scipy.special import expit

import workloads as W


def _random_box(seed, shape=(9, 11, 13), porosity=0.7):
    rng = np.random.default_rng(seed)
    img = (rng.random(shape) < porosity).astype(np.uint8)
    eps = rng.uniform(0.2, 1.5, size=shape)
    return img, eps


def test_constant_factor_is_scaled_d(oracle_mod):
    img, _ = _random_box(1)
    rng = np.random.default_rng(2)
    dirichlet = {(0, 0): 1.0}
    p1 = oracle_mod.Problem(img, [0.4], dirichlet=dirichlet, robin={0: 0.05},
                            reactions=[(0, -1, 0.01)], eps=np.full(img.shape, 2.5))
    p2 = oracle_mod.Problem(img, [1.0], dirichlet=dirichlet, robin={0: 0.05},
                            reactions=[(0, -1, 0.01)])
    c0 = p1.apply_dirichlet(rng.random((1,) + img.shape))
    a = p1.run(c0, 0.05, 40)
    b = p2.run(c0, 0.05, 40)
    assert np.max(np.abs(a - b)) < 1e-14


def test_mass_conserved_with_factor(oracle_mod):
    img, eps = _random_box(3)
    rng = np.random.default_rng(4)
    prob = oracle_mod.Problem(img, [0.8], eps=eps)
    c0 = prob.apply_dirichlet(rng.random((1,) + img.shape))
    m0 = c0.sum()
    c = prob.run(c0, 0.05, 60)
    assert abs(c.sum() - m0) < 1e-12 * m0
    # and the field really moved (the factor is not ignored)
    plain = oracle_mod.Problem(img, [0.8]).run(c0, 0.05, 60)
    assert np.max(np.abs(c - plain)) > 1e-3


def test_discrete_balance_with_factor(oracle_mod):
    img, eps = _random_box(5)
    rng = np.random.default_rng(6)
    prob = oracle_mod.Problem(img, [0.7], dirichlet={(0, 0): 1.0, (0, 5): 0.25},
                              robin={0: 0.03}, reactions=[(0, -1, 0.02)], eps=eps)
    c0 = prob.apply_dirichlet(rng.random((1,) + img.shape))
    dt = 0.05
    m0, inflow, uptake, react = prob.balance(c0, 0)
    c1 = prob.run(c0, dt, 1)
    m1 = prob.balance(c1, 0)[0]
    assert abs((m1 - m0) - dt * (inflow.sum() - uptake + react)) < 1e-12


def _series_steady(w):
    """Exact discrete steady state of a chain with conductances w[i] between i and i+1,
    c = 1 at the first voxel and 0 at the last; and the through-flux."""
    R = np.concatenate([[0.0], np.cumsum(1.0 / w)])
    J = 1.0 / R[-1]
    return 1.0 - J * R, J


@pytest.mark.parametrize("ny,nz", [(1, 1), (3, 2)])
def test_series_conductance_fixed_point(oracle_mod, ny, nz):
    n = 17
    rng = np.random.default_rng(7)
    ex = rng.uniform(0.1, 2.0, size=n)
    eps = np.broadcast_to(ex, (nz, ny, n)).copy()
    img = np.ones((nz, ny, n), dtype=np.uint8)
    D = 0.6
    prob = oracle_mod.Problem(img, [D], dirichlet={(0, 0): 1.0, (0, 1): 0.0}, eps=eps)
    w = D * 0.5 * (ex[:-1] + ex[1:])
    cs, J = _series_steady(w)
    c0 = np.broadcast_to(cs, (1, nz, ny, n)).copy()
    c1 = prob.run(c0, 0.2, 1)
    assert np.max(np.abs(c1 - c0)) < 1e-14
    _, inflow, _, _ = prob.balance(c0, 0)
    area = ny * nz
    assert abs(inflow[0] - J * area) < 1e-13
    assert abs(inflow[1] + J * area) < 1e-13


def test_linear_diffusivity_second_order(oracle_mod):
    errs = []
    for n in (17, 33):
        x = np.linspace(0.0, 1.0, n)
        img = np.ones((1, 1, n), dtype=np.uint8)
        eps = (1.0 + x).reshape(1, 1, n)
        prob = oracle_mod.Problem(img, [1.0], dx=1.0 / (n - 1),
                                  dirichlet={(0, 0): 1.0, (0, 1): 0.0}, eps=eps)
        h = 1.0 / (n - 1)
        dt = 0.2 * h * h  # below h^2 / (2 D_max) = h^2 / 4
        steps = int(12.0 / dt)
        c = prob.run(prob.initial(), dt, steps)[0, 0, 0]
        exact = 1.0 - np.log1p(x) / math.log(2.0)
        errs.append(np.max(np.abs(c - exact)))
    order = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-4
    assert 1.8 < order < 2.2, (errs, order)


def test_smooth_diffusivity(oracle_mod):
    rng = np.random.default_rng(8)
    phi = rng.uniform(-6, 6, size=1000)
    d_min, d_max, g1, g2 = 0.05, 1.3, -0.7, 2.2
    got = oracle_mod.smooth_diffusivity(phi, d_min, d_max, g1, g2)
    ref = d_min + d_max * expit(g1 + g2 * phi)
    assert np.max(np.abs(got - ref)) < 1e-14
    # limits, the transition point, point symmetry about it
    lim = oracle_mod.smooth_diffusivity(np.array([-1e4, 1e4, -g1 / g2]), d_min, d_max, g1, g2)
    assert lim[0] == pytest.approx(d_min, abs=1e-15)
    assert lim[1] == pytest.approx(d_min + d_max, abs=1e-15)
    assert lim[2] == pytest.approx(d_min + d_max / 2, abs=1e-15)
    mirror = -2 * g1 / g2 - phi  # g1 + g2 * mirror = -(g1 + g2 * phi)
    s = got + oracle_mod.smooth_diffusivity(mirror, d_min, d_max, g1, g2)
    assert np.max(np.abs(s - (2 * d_min + d_max))) < 1e-13
    assert np.all(np.diff(oracle_mod.smooth_diffusivity(np.sort(phi), d_min, d_max, g1, g2)) >= 0)


# ---------------------------------------------------------------------------
# volumetric near-surface sink (section "Application example 2": a sink restricted to
# the surface by the level set)
# ---------------------------------------------------------------------------

def test_sink_uniform_closed_form(oracle_mod):
    img = np.ones((6, 7, 8), np.uint8)
    prob = oracle_mod.Problem(img, [1.0], sink={0: 0.3}, sink_mask=np.ones(img.shape, np.uint8))
    c = prob.run(np.full((1,) + img.shape, 2.0), 0.1, 25)
    np.testing.assert_allclose(c, 2.0 * (1 - 0.03) ** 25, rtol=1e-14)


def test_sink_only_on_the_band(oracle_mod):
    rng = np.random.default_rng(21)
    img, _ = _random_box(21)
    mask = (rng.random(img.shape) < 0.3).astype(np.uint8)
    prob = oracle_mod.Problem(img, [0.0, 0.0], sink={1: 0.2}, sink_mask=mask)
    c0 = prob.apply_dirichlet(rng.random((2,) + img.shape))
    c = prob.run(c0, 0.5, 7)
    act = img != 0
    np.testing.assert_array_equal(c[0], c0[0])
    want = np.where(mask != 0, c0[1] * (1 - 0.1) ** 7, c0[1])
    np.testing.assert_allclose(c[1][act], want[act], rtol=1e-14)


def test_sink_in_the_step_balance(oracle_mod):
    img, eps = _random_box(22)
    rng = np.random.default_rng(22)
    mask = (rng.random(img.shape) < 0.4).astype(np.uint8)
    prob = oracle_mod.Problem(img, [0.7], dirichlet={(0, 0): 1.0}, robin={0: 0.03},
                              reactions=[(0, -1, 0.02)], eps=eps, sink={0: 0.15}, sink_mask=mask)
    c0 = prob.apply_dirichlet(rng.random((1,) + img.shape))
    dt = 0.05
    m0, inflow, uptake, react = prob.balance(c0, 0)
    m1 = prob.balance(prob.run(c0, dt, 1), 0)[0]
    assert abs((m1 - m0) - dt * (inflow.sum() - uptake + react)) < 1e-12
    no_sink = oracle_mod.Problem(img, [0.7], dirichlet={(0, 0): 1.0}, robin={0: 0.03},
                                 reactions=[(0, -1, 0.02)], eps=eps)
    act = (img != 0) & (mask != 0)
    act[:, :, 0] = False  # Dirichlet plane
    assert uptake - no_sink.balance(c0, 0)[2] == pytest.approx(0.15 * c0[0][act].sum(), rel=1e-12)


def test_plane_flux_with_factor(oracle_mod):
    """At the series-conductance steady state every plane carries the through-flux; a
    unit factor gives the constant-D flux."""
    n, ny, nz = 17, 3, 2
    rng = np.random.default_rng(30)
    ex = rng.uniform(0.1, 2.0, size=n)
    eps = np.broadcast_to(ex, (nz, ny, n)).copy()
    img = np.ones((nz, ny, n), dtype=np.uint8)
    D = 0.6
    prob = oracle_mod.Problem(img, [D], dirichlet={(0, 0): 1.0, (0, 1): 0.0}, eps=eps)
    cs, J = _series_steady(D * 0.5 * (ex[:-1] + ex[1:]))
    u = np.broadcast_to(cs, (nz, ny, n)).copy()
    for i0 in range(n - 1):
        assert prob.plane_flux(u, D, 0, i0) == pytest.approx(J * ny * nz, rel=1e-12)
    img2, _ = _random_box(31)
    u2 = np.random.default_rng(31).random(img2.shape)
    p1 = oracle_mod.Problem(img2, [0.7], eps=np.ones(img2.shape))
    p0 = oracle_mod.Problem(img2, [0.7])
    for axis in range(3):
        assert p1.plane_flux(u2, 0.7, axis, 4) == pytest.approx(p0.plane_flux(u2, 0.7, axis, 4), rel=1e-14)
