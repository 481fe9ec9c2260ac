"""Checkpointed discrete adjoint on the GPU (through the C ABI) against the FP64
oracle's adjoint, a closed form and torch.autograd."""
import numpy as np
import pytest

import workloads as W
from gpu_common import fields, make_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch

    assert torch.cuda.is_available()
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _case(oracle_mod, n=24, seed=3, steps=120, dt=0.1):
    img, _ = W.boolean_spheres(n, 0.5, 2.0, 4.0, seed=seed)
    img[:, :, 0] = 1
    prob_t = oracle_mod.Problem(img, [1.0], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, 0.01)])
    target = prob_t.run(prob_t.initial(), dt, steps)[0].astype(np.float32)
    return img, target


def _gpu_adjoint(rd, img, target, D, k, dt, steps, every, B=8, storage="fp32"):
    cp = -(-steps // every) + every - 1
    g, s = make_gpu(rd, img, [D], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, k)], B=B,
                    storage=storage, features=rd.RD_WS_ADJOINT, checkpoint_slots=cp)
    return s.adjoint(target, steps, dt, every), s


@pytest.mark.parametrize("B", [8, 4])
def test_adjoint_vs_oracle(rd, oracle_mod, B):
    img, target = _case(oracle_mod)
    D, k, dt, steps = 0.8, 0.02, 0.1, 120
    (L, gD, gk), s = _gpu_adjoint(rd, img, target, D, k, dt, steps, 10, B=B)
    prob = oracle_mod.Problem(img, [D], dirichlet={(0, 0): 1.0})
    c0 = prob.initial()[0]
    Lo, gDo, gko, _ = oracle_mod.adjoint_decay(img, D, k, dt, steps, c0, target.astype(np.float64),
                                               stride=50)
    print(f"B={B}: loss {L:.10e} vs {Lo:.10e}; dL/dD {gD:.10e} vs {gDo:.10e}; dL/dk {gk:.10e} vs "
          f"{gko:.10e}")
    # measured: loss 4.5e-8, gradients 3e-9 relative (FP32 fields, FP64 sums, 120 steps)
    assert L == pytest.approx(Lo, rel=5e-7)
    assert gD == pytest.approx(gDo, rel=1e-7)
    assert gk == pytest.approx(gko, rel=1e-7)


def test_adjoint_checkpoint_stride_bitwise(rd, oracle_mod):
    """Recomputed segment states are bitwise the forward states, so the gradients do
    not depend on the checkpoint stride."""
    img, target = _case(oracle_mod, n=20, seed=5, steps=75)
    res = [_gpu_adjoint(rd, img, target, 0.8, 0.02, 0.1, 75, every)[0] for every in (1, 7, 25, 75)]
    for r in res[1:]:
        assert r == res[0]


def test_adjoint_uniform_closed_form(rd):
    img, _ = W.boolean_spheres(16, 0.5, 2.0, 3.0, seed=2)
    k, dt, N, c0v = 0.02, 0.1, 40, 0.6
    g, s = make_gpu(rd, img, [0.8], reactions=[(0, -1, k)], features=rd.RD_WS_ADJOINT,
                    checkpoint_slots=-(-N // 8) + 7)
    s.set_field(0, (np.where(img != 0, c0v, 0.0)).astype(np.float32))
    target = np.where(img != 0, 0.3, 0.0).astype(np.float32)
    L, gD, gk = s.adjoint(target, N, dt, 8)
    nf = int(img.sum())
    cN = c0v * (1 - k * dt) ** N
    # L c^n = 0 for a uniform field; in FP32 the six-neighbour sum of equal values can be
    # an ulp off, which the update (increment form) keeps, so dL/dD is round-off
    assert abs(gD) <= 1e-9 * abs(gk)
    assert gk == pytest.approx(-nf * (cN - 0.3) * c0v * N * dt * (1 - k * dt) ** (N - 1), rel=1e-5)
    assert L == pytest.approx(0.5 * nf * (cN - 0.3) ** 2, rel=1e-5)


def test_decay_workload_reduced(rd, oracle_mod):
    """Diffusion-decay recipe at 64^3 (p = 0.5), D = 0.8, k = 0.02, 2000 steps,
    checkpoints every 100 steps, target from D = 1, k = 0.01."""
    w = W.workload("decay256", small=True)
    img, _ = W.workload_geometry("decay256", small=True)
    prob_t = oracle_mod.Problem(img, [1.0], dirichlet=w.dirichlet, reactions=[(0, -1, 0.01)])
    target = prob_t.run(prob_t.initial(), w.dt, w.steps)[0].astype(np.float32)
    (L, gD, gk), _ = _gpu_adjoint(rd, img, target, 0.8, 0.02, w.dt, w.steps, 100)
    prob = oracle_mod.Problem(img, [0.8], dirichlet=w.dirichlet)
    Lo, gDo, gko, _ = oracle_mod.adjoint_decay(img, 0.8, 0.02, w.dt, w.steps, prob.initial()[0],
                                               target.astype(np.float64), stride=50)
    print(f"decay64: loss {L:.10e}/{Lo:.10e} dD {gD:.10e}/{gDo:.10e} dk {gk:.10e}/{gko:.10e}")
    # measured: loss 1.2e-6, dL/dD 6e-7, dL/dk < 4e-7 relative after 2000 FP32 steps
    assert L == pytest.approx(Lo, rel=5e-6)
    assert gD == pytest.approx(gDo, rel=3e-6)
    assert gk == pytest.approx(gko, rel=3e-6)


def test_autograd_function(rd, oracle_mod):
    import torch

    img, target = _case(oracle_mod, n=16, seed=7, steps=60)
    D0, k0, dt, steps = 0.8, 0.02, 0.1, 60
    cp = -(-steps // 20) + 19
    g, s = make_gpu(rd, img, [D0], dirichlet={(0, 0): 1.0}, reactions=[(0, -1, k0)],
                    features=rd.RD_WS_ADJOINT, checkpoint_slots=cp)
    c0 = fields(s, 1)[0].astype(np.float32)
    c0t = torch.tensor(c0, device="cuda")
    tgt = torch.tensor(target, device="cuda")
    D = torch.tensor(D0, dtype=torch.float64, requires_grad=True)
    k = torch.tensor(k0, dtype=torch.float64, requires_grad=True)
    cN = rd.DiffusionDecay.apply(D, k, s, c0t, steps, dt, 20)
    free = torch.tensor(img != 0, device="cuda")
    free[:, :, 0] = False  # Dirichlet plane
    loss = 0.5 * (((cN - tgt) * free) ** 2).sum()
    loss.backward()
    s.set_field(0, c0t)
    L, gD, gk = s.adjoint(target, steps, dt, 20)
    assert D.grad.item() == pytest.approx(gD, rel=1e-6)
    assert k.grad.item() == pytest.approx(gk, rel=1e-6)
    assert loss.item() == pytest.approx(L, rel=1e-5)
