"""Pins of the oracle's UNO preconditioner and its second-order training for
three nodal DOF (App. B): the local parametrization against its printed
matrix, reduction to the one-DOF preconditioner for isotropic weights, the
spectrum lemma of Sec. 4.2.3 on a dense matrix, the feature loss against the
sample loss, derivatives against finite differences, Newton training that
recovers a planted preconditioner, and UNO-CG on an elastic problem."""
import numpy as np
import pytest

import synth_inputs as si


def test_psi3_matches_printed_matrix_and_is_spd(orc):
    rng = np.random.default_rng(1)
    for _ in range(5):
        w1, w2, w3, w4, w5, w6 = w = rng.standard_normal(6)
        P = np.array([[w1 * w1, w1 * w3, w1 * w6],
                      [w1 * w3, w2 * w2 + w3 * w3, w2 * w5 + w3 * w6],
                      [w1 * w6, w2 * w5 + w3 * w6, w4 * w4 + w5 * w5 + w6 * w6]])
        Q = orc.q_matrix(orc.psi3(w))
        assert np.abs(Q - P).max() < 1e-14 * np.abs(P).max()
        assert np.linalg.eigvalsh(Q).min() > 0.0


def _iso_theta(th1):
    th = np.zeros(6 * th1.size)
    th.reshape(-1, 6)[:, [0, 1, 3]] = th1[:, None]
    return th


@pytest.mark.parametrize("shape,M", [((6, 5, 7), 1), ((8, 8, 6), 2)])
def test_isotropic_weights_reduce_to_one_dof(orc, shape, M):
    """With w = (t, t, 0, t, 0, 0) in every slot, psi = t^2 I and the c = 3
    preconditioner is the c = 1 one with weights t on each component."""
    th1 = si.random_theta(orc.num_weights(3, M), 3)
    th3 = _iso_theta(th1)
    r = np.stack([si.random_field(shape, 10 + c) for c in range(3)])
    s = orc.uno3_apply(orc.uno3_table(shape, M, th3), r)
    for c in range(3):
        assert np.abs(s[c] - orc.uno_apply(th1, M, r[c])).max() < 1e-13 * np.abs(s).max()


@pytest.mark.parametrize("shape,M", [((3, 4, 5), 1), ((4, 4, 3), 1)])
def test_uno3_spectrum_lemma_symmetry_realness(orc, shape, M):
    """eig(P) is the union of the eigenvalues of the 3 x 3 blocks Phi(k)
    (Lemma of Sec. 4.2.3); P is symmetric and maps real to real."""
    rng = np.random.default_rng(5)
    th = rng.standard_normal(orc.num_weights3(M))
    tab = orc.uno3_table(shape, M, th)
    n = int(np.prod(shape))
    P = np.zeros((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n)
        e[j] = 1.0
        P[:, j] = orc.uno3_apply(tab, e.reshape((3,) + shape)).ravel()
    assert np.abs(P - P.T).max() < 1e-13 * np.abs(P).max()
    blocks = tab.reshape(6, -1).T
    ev = np.concatenate([np.linalg.eigvalsh(orc.q_matrix(q)) for q in blocks])
    assert np.abs(np.sort(np.linalg.eigvalsh(P)) - np.sort(ev)).max() < 1e-12 * np.abs(ev).max()
    s, im = orc.uno3_apply(tab, rng.standard_normal((3,) + shape), return_imag=True)
    assert im < 1e-13 * np.abs(s).max()


def _pairs(orc, shape, rng, ns=4):
    fs = [rng.standard_normal((3,) + shape) for _ in range(ns)]
    us = [rng.standard_normal((3,) + shape) for _ in range(ns)]
    return fs, us


def test_feature_loss_equals_sample_loss(orc):
    shape, M = (6, 5, 6), 1
    rng = np.random.default_rng(7)
    fs, us = _pairs(orc, shape, rng)
    a, b, dl = orc.train3_features(fs, us)
    for _ in range(2):
        th = 0.5 * rng.standard_normal(orc.num_weights3(M))
        tab = orc.uno3_table(shape, M, th)
        direct = np.mean([np.sum((orc.uno3_apply(tab, f) - u) ** 2) for f, u in zip(fs, us)])
        assert orc.train3_loss(th, M, a, b, dl) == pytest.approx(direct, rel=1e-11)


def test_gradient_and_hessian_match_finite_differences(orc):
    shape, M = (5, 5, 4), 1
    rng = np.random.default_rng(8)
    fs, us = _pairs(orc, shape, rng, 3)
    a, b, dl = orc.train3_features(fs, us)
    th = 0.7 * rng.standard_normal(orc.num_weights3(M))
    g, H = orc.train3_grad_hess(th, M, a, b)
    h = 1e-5
    idx = rng.choice(th.size, 24, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (orc.train3_loss(th + e, M, a, b, dl) - orc.train3_loss(th - e, M, a, b, dl)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-8 * np.abs(g).max())
        gd = (orc.train3_grad_hess(th + e, M, a, b, False) - orc.train3_grad_hess(th - e, M, a, b, False)) / (2 * h)
        assert np.abs(gd - H[:, i]).max() < 1e-6 * np.abs(H).max()
    assert np.abs(H - H.T).max() < 1e-12 * np.abs(H).max()


def test_newton_recovers_planted_preconditioner(orc):
    """Targets u = P* f of a known SPD table: the trained table equals it and
    the loss vanishes (the optimal table is unique)."""
    shape, M = (6, 6, 5), 1
    rng = np.random.default_rng(9)
    nw = orc.num_weights3(M)
    th_star = rng.standard_normal(nw)
    th_star.reshape(-1, 6)[:, [0, 1, 3]] += 2.0
    tab_star = orc.uno3_table(shape, M, th_star)
    fs = [rng.standard_normal((3,) + shape) for _ in range(4)]
    us = [orc.uno3_apply(tab_star, f) for f in fs]
    a, b, dl = orc.train3_features(fs, us)
    th, losses = orc.train3_newton(M, a, b, dl, epochs=200)
    assert losses[-1] < 1e-18 * dl
    tab = orc.uno3_table(shape, M, th)
    assert np.abs(tab - tab_star).max() < 1e-7 * np.abs(tab_star).max()


def test_trained_uno3_cg_solves_elastic_problem(orc):
    """UNO-CG with a table trained on solver pairs reaches the Jacobi-CG
    solution in fewer passes (Algorithm 2 for c = 3)."""
    shape, M = (8, 8, 8), 2
    ph, _ = si.rsa_inclusions(shape, 1.0, 2.0, 0.25, 21)
    lam, mu = orc.lame(si.two_phase_kappa(ph, 1.0, 10.0), 0.3)
    fs, us = [], []
    for j in range(6):
        f = orc.el_rhs(lam, mu, np.eye(6)[j])
        u, _ = orc.el_pcg(lam, mu, f, "jacobi", rtol=1e-12)
        fs.append(f)
        us.append(u)
    a, b, dl = orc.train3_features(fs, us)
    th, losses = orc.train3_newton(M, a, b, dl, epochs=60)
    assert losses[-1] < losses[0]
    tab = orc.uno3_table(shape, M, th)
    f = orc.el_rhs(lam, mu, np.array([0.3, -0.2, 0.1, 0.4, 0.0, -0.5]))
    uj, itj = orc.el_pcg(lam, mu, f, "jacobi", rtol=1e-10)
    uu, itu = orc.el_pcg(lam, mu, f, "uno", rtol=1e-10, table=tab)
    assert np.abs(uu - uj).max() < 1e-7 * np.abs(uj).max()
    assert itu < itj
