"""Pins of the oracle's discrete adjoint with a per-voxel diffusivity factor: every
gradient against central differences of the oracle's own forward loss, and the
constant-factor case against the pinned constant-D adjoint."""
import numpy as np
import pytest


def _case(seed=3, shape=(5, 6, 7)):
    rng = np.random.default_rng(seed)
    img = (rng.random(shape) < 0.75).astype(np.uint8)
    eps = rng.uniform(0.3, 1.4, size=shape)
    c0 = rng.random(shape)
    c0[:, :, 0] = 1.0  # Dirichlet data on -x
    tgt = rng.random(shape)
    return img, eps, c0, tgt


def test_gradients_match_central_differences(oracle_mod):
    img, eps, c0, tgt = _case()
    D, k, dt, n = 0.7, 0.05, 0.08, 15
    L, gD, gk, ge, _ = oracle_mod.adjoint_factor(img, D, k, eps, dt, n, c0, tgt)

    def loss(D=D, k=k, eps=eps):
        return oracle_mod.adjoint_factor(img, D, k, eps, dt, n, c0, tgt)[0]

    h = 1e-6
    assert gD == pytest.approx((loss(D=D + h) - loss(D=D - h)) / (2 * h), rel=1e-6)
    assert gk == pytest.approx((loss(k=k + h) - loss(k=k - h)) / (2 * h), rel=1e-6)
    act = np.argwhere(img != 0)
    picks = [tuple(p) for p in act[:: max(1, len(act) // 12)]]
    picks += [tuple(p) for p in act if p[2] == 0][:2]  # Dirichlet voxels
    for p in picks:
        ep, em = eps.copy(), eps.copy()
        ep[p] += h
        em[p] -= h
        fd = (loss(eps=ep) - loss(eps=em)) / (2 * h)
        assert ge[p] == pytest.approx(fd, rel=1e-5, abs=1e-11), p
    assert np.all(ge[img == 0] == 0)


def test_constant_factor_matches_constant_d_adjoint(oracle_mod):
    img, _, c0, tgt = _case(seed=5)
    D, k, dt, n = 0.5, 0.02, 0.1, 20
    L1, gD1, gk1, ge, cN1 = oracle_mod.adjoint_factor(img, D, k, np.ones(img.shape), dt, n, c0, tgt)
    L2, gD2, gk2, cN2 = oracle_mod.adjoint_decay(img, D, k, dt, n, c0 * (img != 0), tgt, stride=7)
    assert L1 == pytest.approx(L2, rel=1e-12)
    assert gD1 == pytest.approx(gD2, rel=1e-10)
    assert gk1 == pytest.approx(gk2, rel=1e-10)
    # e = 1 everywhere: scaling e by s scales D by s, so sum_p e_p dL/de_p = D dL/dD
    assert float(np.sum(ge)) == pytest.approx(D * gD1, rel=1e-10)
