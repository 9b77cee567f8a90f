"""Pins of the oracle's second-order training (Sec. 4.4, one nodal DOF):
feature-based loss equals the sample loss of eq. (fnocg-loss), and the
closed-form minimiser is the global optimum found by a library optimiser."""
import numpy as np
import pytest
import scipy.optimize

import synth_inputs as si


def make_pairs(orc, shape, seeds, vf=0.3):
    fs, us = [], []
    for s in seeds:
        ph, _ = si.rsa_inclusions(shape, 1.5, 2.5, vf, s)
        kap = si.two_phase_kappa(ph, 1.0, 10.0)
        for g in np.eye(len(shape)):
            f = orc.rhs(kap, g)
            u, it, hist, fr = orc.pcg(kap, f, "jacobi", rtol=1e-12)
            fs.append(f)
            us.append(u)
    return fs, us


@pytest.fixture(scope="module")
def pairs2d(orc):
    return make_pairs(orc, (10, 10), [1, 2, 3])


def test_feature_loss_equals_sample_loss(orc, pairs2d):
    """L = (1/Ns) sum_j ||P f_j - u_j||^2 equals alpha.(v o v) - beta.v + delta."""
    fs, us = pairs2d
    a, b, dl = orc.train_features(fs, us)
    M = 2
    for seed in (1, 2):
        th = si.random_theta(orc.num_weights(2, M), seed, scale=0.05)
        direct = np.mean([np.sum((orc.uno_apply(th, M, f) - u) ** 2) for f, u in zip(fs, us)])
        assert orc.train_loss(th, M, a, b, dl) == pytest.approx(direct, rel=1e-10)


def test_features_are_even_for_real_data(orc, pairs2d):
    fs, us = pairs2d
    a, b, dl = orc.train_features(fs, us)
    refl = lambda x: np.roll(np.flip(x, axis=(0, 1)), 1, axis=(0, 1))  # k -> -k
    assert np.allclose(a, refl(a), atol=1e-14 * a.max())
    assert np.allclose(b, refl(b), atol=1e-14 * np.abs(b).max())


@pytest.mark.parametrize("M", [1, 2, 3])
def test_closed_form_is_global_minimum(orc, pairs2d, M):
    fs, us = pairs2d
    a, b, dl = orc.train_features(fs, us)
    th = orc.train_closed_form(M, a, b)
    L = orc.train_loss(th, M, a, b, dl)
    # library optimiser over v = theta^2 >= 0 (bounded quasi-Newton)
    nw = orc.num_weights(2, M)
    fun = lambda v: orc.train_loss(np.sqrt(np.maximum(v, 0)), M, a, b, dl)
    v0 = np.full(nw, np.median(np.abs(th)) ** 2 + 1e-3)
    res = scipy.optimize.minimize(fun, v0, method="L-BFGS-B", bounds=[(0, None)] * nw,
                                  options=dict(maxiter=20000, ftol=1e-15, gtol=1e-14))
    assert L <= res.fun + 1e-9 * abs(res.fun)
    # no random perturbation improves it
    rng = np.random.default_rng(0)
    for _ in range(20):
        t2 = th + 1e-3 * np.abs(th).max() * rng.standard_normal(nw)
        assert orc.train_loss(t2, M, a, b, dl) >= L - 1e-12 * abs(L)


def test_trained_preconditioner_beats_jacobi(orc):
    """A UNO trained on solver-generated pairs needs far fewer iterations
    than Jacobi-CG on an unseen microstructure (Sec. 6.1 behaviour)."""
    shape = (16, 16)
    fs, us = make_pairs(orc, shape, list(range(10, 18)))
    a, b, dl = orc.train_features(fs, us)
    M = 4
    th = orc.train_closed_form(M, a, b)
    tab = orc.uno_table(shape, M, th)
    ph, _ = si.rsa_inclusions(shape, 1.5, 2.5, 0.3, 99)
    kap = si.two_phase_kappa(ph, 1.0, 10.0)
    f = orc.rhs(kap, [1.0, 0.0])
    _, it_uno, _, _ = orc.pcg(kap, f, "uno", table=tab, rtol=1e-6)
    _, it_jac, _, _ = orc.pcg(kap, f, "jacobi", rtol=1e-6)
    assert it_uno * 2 < it_jac
