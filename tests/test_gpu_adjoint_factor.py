"""Discrete adjoint with a per-voxel diffusivity factor on the GPU (through the C ABI)
against the oracle's, including dL/de per voxel and the chain rule to the parameters of
the smooth D(phi)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import make_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _case(oracle_mod, n=22, seed=7, steps=80, dt=0.06):
    img, _ = W.boolean_spheres(n, 0.5, 2.0, 4.0, seed=seed)
    img[:, :, 0] = 1
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.3, 1.4, img.shape).astype(np.float32).astype(np.float64)
    prob_t = oracle_mod.Problem(img, [1.0], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, 0.01)])
    target = prob_t.run(prob_t.initial(), dt, steps)[0].astype(np.float32)
    return img, eps, target


def _gpu(rd, img, eps, target, D, k, dt, steps, every, B=8, kernel="column"):
    cp = -(-steps // every) + every - 1
    _, s = make_gpu(rd, img, [D], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, k)], B=B, kernel=kernel,
                    features=rd.RD_WS_ADJOINT | rd.RD_WS_DIFFUSIVITY, checkpoint_slots=cp)
    s.set_diffusivity(eps.astype(np.float32))
    L, gD, gk, ge = s.adjoint_factor(target, steps, dt, every)
    return (L, gD, gk, ge.cpu().numpy()), s


@pytest.mark.parametrize("B,kernel", [(8, "column"), (4, "block")])
def test_vs_oracle(rd, oracle_mod, B, kernel):
    img, eps, target = _case(oracle_mod)
    D, k, dt, steps = 0.8, 0.02, 0.06, 80
    (L, gD, gk, ge), _ = _gpu(rd, img, eps, target, D, k, dt, steps, 10, B=B, kernel=kernel)
    c0 = oracle_mod.Problem(img, [D], dirichlet={(0, 0): 1.0}).initial()[0]
    Lo, gDo, gko, geo, _ = oracle_mod.adjoint_factor(img, D, k, eps, dt, steps, c0,
                                                    target.astype(np.float64))
    err = rel_l2(ge, geo, img != 0)
    print(f"B={B}: loss {L:.8e} vs {Lo:.8e}; dL/dD {gD:.8e} vs {gDo:.8e}; dL/dk {gk:.8e} vs "
          f"{gko:.8e}; dL/de rel L2 {err:.2e}")
    # measured: loss 1.3e-7, dL/dD 8.5e-8, dL/dk 8.2e-8, dL/de 2.35e-7 relative
    assert L == pytest.approx(Lo, rel=1e-6)
    assert gD == pytest.approx(gDo, rel=5e-7)
    assert gk == pytest.approx(gko, rel=5e-7)
    assert err < 1e-6
    assert np.all(ge[img == 0] == 0)


def test_checkpoint_stride_bitwise(rd, oracle_mod):
    img, eps, target = _case(oracle_mod, n=18, seed=9, steps=45)
    res = [_gpu(rd, img, eps, target, 0.8, 0.02, 0.06, 45, every)[0] for every in (1, 7, 45)]
    for r in res[1:]:
        assert r[:3] == res[0][:3]
        assert np.array_equal(r[3], res[0][3])


def test_chain_rule_to_smooth_d_parameters(rd, oracle_mod):
    """dL/dg1 and dL/dg2 from the GPU's dL/de and the derivative of D(phi) == central
    differences (h = 1e-3) of the FP64 oracle's loss in g1 and g2."""
    import torch

    img, _, target = _case(oracle_mod, n=20, seed=11, steps=60)
    phi = oracle_mod.signed_distance(img, 1.0)
    d_min, d_max, g1, g2 = 0.1, 0.9, -2.0, 2.0
    dt, steps = 0.08, 60
    _, s = make_gpu(rd, img, [1.0], dirichlet={(0, 0): 1.0}, kernel="column",
                    features=rd.RD_WS_ADJOINT | rd.RD_WS_DIFFUSIVITY, checkpoint_slots=20)
    s.set_diffusivity_sdf(phi, d_min, d_max, g1, g2)
    _, _, _, ge = s.adjoint_factor(target, steps, dt, 10)
    ph = torch.as_tensor(phi.astype(np.float64), device=ge.device)
    sig = torch.sigmoid(g1 + g2 * ph)
    dg1 = float(torch.sum(ge * d_max * sig * (1 - sig)))
    dg2 = float(torch.sum(ge * d_max * sig * (1 - sig) * ph))

    def oracle_loss(g1_, g2_):
        eps = oracle_mod.smooth_diffusivity(phi.astype(np.float64), d_min, d_max, g1_, g2_)
        prob = oracle_mod.Problem(img, [1.0], dirichlet={(0, 0): 1.0}, eps=eps)
        cN = prob.run(prob.initial(), dt, steps)[0]
        d = (cN - target.astype(np.float64))[prob.free_mask(0)]
        return 0.5 * float(np.sum(d * d))

    h = 1e-3
    fd1 = (oracle_loss(g1 + h, g2) - oracle_loss(g1 - h, g2)) / (2 * h)
    fd2 = (oracle_loss(g1, g2 + h) - oracle_loss(g1, g2 - h)) / (2 * h)
    print(f"dL/dg1 adjoint {dg1:.10e} FP64 central differences {fd1:.10e} (rel "
          f"{abs(dg1 - fd1) / abs(fd1):.2e}); dL/dg2 {dg2:.10e} vs {fd2:.10e} (rel "
          f"{abs(dg2 - fd2) / abs(fd2):.2e})")
    assert dg1 == pytest.approx(fd1, rel=1e-4)
    assert dg2 == pytest.approx(fd2, rel=1e-4)


def test_errors(rd, oracle_mod):
    img, eps, target = _case(oracle_mod, n=12, steps=5)
    _, s = make_gpu(rd, img, [1.0], features=rd.RD_WS_ADJOINT | rd.RD_WS_DIFFUSIVITY, checkpoint_slots=8)
    with pytest.raises(rd.RDError) as ex:
        s.adjoint_factor(target, 5, 0.05, 5)  # no factor set
    assert ex.value.name == "RD_ERR_STATE"
    _, s2 = make_gpu(rd, img, [1.0], features=rd.RD_WS_ADJOINT, checkpoint_slots=8)
    with pytest.raises(rd.RDError) as ex:
        s2.adjoint_factor(target, 5, 0.05, 5)
    assert ex.value.name == "RD_ERR_WORKSPACE"


def test_column_and_per_slot_kernels_agree(rd, oracle_mod):
    """B = 8: the column adjoint kernel and the one-thread-per-slot kernel give the same
    dL/de bits; the gradient rows are summed in another order."""
    img, eps, target = _case(oracle_mod, n=26, seed=13, steps=40)
    col = _gpu(rd, img, eps, target, 0.8, 0.02, 0.06, 40, 10, kernel="column")[0]
    per = _gpu(rd, img, eps, target, 0.8, 0.02, 0.06, 40, 10, kernel="block")[0]
    assert np.array_equal(col[3], per[3])
    assert col[0] == per[0]
    assert col[1] == pytest.approx(per[1], rel=1e-12)
    assert col[2] == pytest.approx(per[2], rel=1e-12)
