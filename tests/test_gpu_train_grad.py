"""GPU: first-order training step of the UNO weights (Algorithm 3) — loss and
hand-written gradient against the oracle's loss (central differences), zero
gradient at the oracle's exact minimiser, and Adam steps on the autograd
wrapper that approach that minimum; then one step at 64^3 on a batch of 16
pairs solved on the GPU."""
import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def uno():
    import paper_2508_02681_amd as u
    u.lib()
    assert torch.cuda.is_available()
    return u


def _pairs(orc, shape, ns, seed):
    fs, us = [], []
    for j in range(ns):
        ph, _ = si.rsa_inclusions(shape, 1 if min(shape) < 12 else 2, 2 if min(shape) < 12 else 4, 0.3, seed + j)
        kap = si.two_phase_kappa(ph, 1.0, 10.0)
        g = np.zeros(len(shape))
        g[j % len(shape)] = 1.0
        f = orc.rhs(kap, g)
        fs.append(f)
        us.append(orc.pcg(kap, f, "jacobi", rtol=1e-12)[0])
    return fs, us


def _half(a):
    n = a.shape[-1]
    return np.ascontiguousarray(a[..., : n // 2 + 1])


@pytest.mark.parametrize("shape,M", [((16, 16), 3), ((12, 10, 8), 2)])
def test_loss_and_gradient_match_oracle(orc, uno, shape, M):
    fs, us = _pairs(orc, shape, 4, 60)
    A, B, delta = orc.train_features(fs, us)
    At = torch.tensor(_half(A), device=DEV)
    Bt = torch.tensor(_half(B), device=DEV)
    rng = np.random.default_rng(61)
    nw = uno.num_weights(len(shape), M)
    th = np.abs(rng.standard_normal(nw)) * 0.05 + 0.01
    loss, grad = uno.uno_train_loss_grad(shape, M, At, Bt, th)
    ref = orc.train_loss(th, M, A, B, delta) - delta
    assert abs(loss - ref) < 1e-12 * (abs(ref) + delta)
    fd = np.zeros(nw)
    for i in range(nw):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (orc.train_loss(tp, M, A, B, delta) - orc.train_loss(tm, M, A, B, delta)) / (2 * h)
    assert np.abs(grad - fd).max() < 1e-6 * np.abs(fd).max()


def test_gradient_vanishes_at_exact_minimiser(orc, uno):
    shape, M = (16, 16), 3
    fs, us = _pairs(orc, shape, 6, 62)
    A, B, delta = orc.train_features(fs, us)
    th = orc.train_closed_form(M, A, B)
    _, grad = uno.uno_train_loss_grad(shape, M, torch.tensor(_half(A), device=DEV), torch.tensor(_half(B), device=DEV), th)
    _, g0 = uno.uno_train_loss_grad(shape, M, torch.tensor(_half(A), device=DEV), torch.tensor(_half(B), device=DEV),
                                    th * 1.1)
    assert np.abs(grad).max() < 1e-9 * np.abs(g0).max()


def test_adam_steps_on_autograd_wrapper_approach_minimum(orc, uno):
    shape, M = (16, 16), 3
    fs, us = _pairs(orc, shape, 6, 63)
    A, B, delta = orc.train_features(fs, us)
    At, Bt = torch.tensor(_half(A), device=DEV), torch.tensor(_half(B), device=DEV)
    best = orc.train_loss(orc.train_closed_form(M, A, B), M, A, B, delta) - delta
    nw = uno.num_weights(2, M)
    theta = torch.tensor(si.random_theta(nw, 64, scale=0.3, spread=0.1), dtype=torch.float64,
                         device=DEV).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=0.01)
    losses = []
    for _ in range(400):
        opt.zero_grad()
        L = uno.UnoTrainLoss.apply(theta, shape, M, At, Bt)
        L.backward()
        opt.step()
        losses.append(float(L.detach()))
    assert losses[-1] < losses[0]
    assert losses[-1] - best < 0.05 * (losses[0] - best)


def test_training_step_64cubed_batch16(uno):
    """The 64^3 workload: 16 training pairs (4 microstructures x ... loads)
    solved by GPU UNO-CG from a random start, features, one gradient step."""
    cfg = dict(si.CONFIG_3D_64)
    shape = (64, 64, 64)
    M = 8
    nw = uno.num_weights(3, M)
    theta = si.random_theta(nw, 65, scale=0.08, spread=0.1)
    p = uno.UnoPrecond.create(shape, M, theta)
    F, U = [], []
    for s in range(6):
        kap = torch.tensor(si.microstructure(cfg, s)[0], device=DEV)
        u, infos = uno.pcg_solve_batch(kap, macro_loads=np.eye(3), kind="uno", precond=p, rtol=1e-8)
        assert all(i["converged"] for i in infos)
        for j in range(3):
            F.append(uno.uno_macro_rhs(kap, np.eye(3)[j]))
            U.append(u[j])
    F, U = torch.stack(F[:16]), torch.stack(U[:16])
    A = torch.zeros(uno.half_shape(shape), dtype=torch.float64, device=DEV)
    B = torch.zeros_like(A)
    uno.uno_train_accumulate(F, U, A, B, 16)
    th = torch.tensor(theta, dtype=torch.float64, device=DEV).requires_grad_(True)
    L0 = uno.UnoTrainLoss.apply(th, shape, M, A, B)
    L0.backward()
    g = th.grad.detach()
    step = 0.5 * float(th.detach().abs().mean()) / float(g.abs().max())
    with torch.no_grad():
        th2 = th - step * g
    L1 = uno.UnoTrainLoss.apply(th2, shape, M, A, B)
    assert float(L1) < float(L0)
