"""GPU: second-order training of the UNO weights for three nodal DOF (App. B)
against the oracle: features on the half spectrum, Newton training to the
same optimal table, recovery of a planted preconditioner, and UNO-CG with
trained weights beating Jacobi-CG."""
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


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def gpu_features(uno, shape, fs, us):
    nh = shape[2] // 2 + 1
    A = torch.zeros((6, shape[0], shape[1], nh), dtype=torch.float64, device=DEV)
    B = torch.zeros_like(A)
    F, U = T(np.stack(fs)), T(np.stack(us))
    half = len(fs) // 2  # two calls: accumulation over batches
    uno.el_uno_train_accumulate(F[:half], U[:half], A, B, len(fs))
    uno.el_uno_train_accumulate(F[half:], U[half:], A, B, len(fs))
    return A, B


def test_features_match_oracle(orc, uno):
    shape = (6, 8, 10)
    rng = np.random.default_rng(40)
    fs = [rng.standard_normal((3,) + shape) for _ in range(5)]
    us = [rng.standard_normal((3,) + shape) for _ in range(5)]
    A, B = gpu_features(uno, shape, fs, us)
    a, b, _ = orc.train3_features(fs, us)
    nh = shape[2] // 2 + 1
    for x, y in ((A, a), (B, b)):
        ref = y[..., :nh]
        assert np.abs(x.cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()


def test_fit_recovers_planted_preconditioner(orc, uno):
    shape, M = (6, 6, 6), 1
    rng = np.random.default_rng(41)
    th_star = rng.standard_normal(orc.num_weights3(M))
    th_star.reshape(-1, 6)[:, [0, 1, 3]] += 2.0
    tab_star = orc.uno3_table(shape, M, th_star)
    fs = [rng.standard_normal((3,) + shape) for _ in range(4)]
    us = [orc.uno3_apply(tab_star, f) for f in fs]
    A, B = gpu_features(uno, shape, fs, us)
    _, _, dl = orc.train3_features(fs, us)
    th, loss = uno.el_uno_train_fit(shape, M, A, B)
    assert abs(loss + dl) < 1e-12 * dl  # the loss less delta cancels delta to rounding
    assert np.abs(orc.uno3_table(shape, M, th) - tab_star).max() < 1e-7 * np.abs(tab_star).max()


def _elastic_pairs(orc, shape, seed):
    ph, _ = si.rsa_inclusions(shape, 1.0, 2.0, 0.25, seed)
    lam, mu = orc.lame(si.two_phase_kappa(ph, 1.0, 10.0), 0.3)
    fs, us = [], []
    for j in range(6):
        f = orc.el_rhs(lam, mu, np.eye(6)[j])
        u, _ = orc.el_pcg(lam, mu, f, "jacobi", rtol=1e-12)
        fs.append(f)
        us.append(u)
    return lam, mu, fs, us


def test_fit_reaches_the_oracle_optimum(orc, uno):
    """Solver pairs: the optimal table is unique, so the trained tables and
    losses of both agree (the oracle trains every slot, the library ties the
    two slots of a k_z = 0 pair)."""
    shape, M = (8, 8, 8), 2
    lam, mu, fs, us = _elastic_pairs(orc, shape, 42)
    A, B = gpu_features(uno, shape, fs, us)
    a, b, dl = orc.train3_features(fs, us)
    th, loss = uno.el_uno_train_fit(shape, M, A, B)
    tho, losses = orc.train3_newton(M, a, b, dl, epochs=200)
    assert loss + dl == pytest.approx(losses[-1], rel=1e-9)
    assert orc.train3_loss(th, M, a, b, dl) == pytest.approx(losses[-1], rel=1e-9)
    t1, t2 = orc.uno3_table(shape, M, th), orc.uno3_table(shape, M, tho)
    assert np.abs(t1 - t2).max() < 1e-4 * np.abs(t2).max()


def test_trained_uno_cg_beats_jacobi_on_gpu(orc, uno):
    shape, M = (16, 16, 16), 3
    rng = np.random.default_rng(43)
    fs, us = [], []
    for seed in (44, 45):
        ph, _ = si.rsa_inclusions(shape, 2.0, 4.0, 0.25, seed)
        lam, mu = orc.lame(si.two_phase_kappa(ph, 1.0, 10.0), 0.3)
        u, _ = uno.el_pcg_solve(T(lam), T(mu), np.eye(6), rtol=1e-10)
        for j in range(6):
            fs.append(uno.el_macro_rhs(T(lam), T(mu), np.eye(6)[j]))
            us.append(u[j])
    nh = shape[2] // 2 + 1
    A = torch.zeros((6, shape[0], shape[1], nh), dtype=torch.float64, device=DEV)
    B = torch.zeros_like(A)
    uno.el_uno_train_accumulate(torch.stack(fs), torch.stack(us), A, B, len(fs))
    th, _ = uno.el_uno_train_fit(shape, M, A, B)
    P = uno.UnoPrecond.create_elastic(shape, M, th)
    ph, _ = si.rsa_inclusions(shape, 2.0, 4.0, 0.25, 46)
    lam, mu = orc.lame(si.two_phase_kappa(ph, 1.0, 10.0), 0.3)
    loads = rng.standard_normal((3, 6))
    uj, ij = uno.el_pcg_solve(T(lam), T(mu), loads, rtol=1e-8)
    uu, iu = uno.el_pcg_solve(T(lam), T(mu), loads, kind="uno", precond=P, rtol=1e-8)
    for a, b in zip(ij, iu):
        assert b["converged"] and b["iters"] < a["iters"]
    assert (uu - uj).abs().max().item() < 1e-6 * uj.abs().max().item()
