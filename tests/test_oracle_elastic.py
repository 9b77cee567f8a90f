"""Pins of the oracle's 3D linear-elasticity path (Sec. 5.2, c = 3, Mandel
basis of App. A): element matrix rigid-body null space and exact energy of a
uniform strain, periodic operator symmetry and translation null space,
homogeneous medium, exact laminate stiffnesses (harmonic and arithmetic
means), Voigt/Reuss bounds, and a dense bordered direct solve."""
import numpy as np
import pytest

import synth_inputs as si

SQ2 = np.sqrt(2.0)


def _mandel(eps33):
    e = eps33
    return np.array([e[0, 0], e[1, 1], e[2, 2], SQ2 * e[0, 1], SQ2 * e[0, 2], SQ2 * e[1, 2]])


def _D(lam, mu):
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    return D + 2 * mu * np.eye(6)


def _corner_xyz(h):
    return np.array([[(a >> 2) & 1, (a >> 1) & 1, a & 1] for a in range(8)], dtype=float) * np.asarray(h)


@pytest.mark.parametrize("lam,mu", [(1.0, 0.0), (0.0, 1.0), (2.3, 0.7)])
def test_element_matrix_rigid_modes_and_uniform_strain_energy(orc, lam, mu):
    shape = (4, 5, 6)
    h = [1.0 / s for s in shape]
    K = orc.el_element_matrix(shape, lam, mu)
    assert np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    X = _corner_xyz(h)
    modes = []
    for c in range(3):  # translations
        v = np.zeros((8, 3)); v[:, c] = 1.0; modes.append(v.ravel())
    for (a, b) in [(0, 1), (0, 2), (1, 2)]:  # infinitesimal rotations
        v = np.zeros((8, 3)); v[:, a] = -X[:, b]; v[:, b] = X[:, a]; modes.append(v.ravel())
    for v in modes:
        assert np.abs(K @ v).max() < 1e-12 * np.abs(K).max()
    rng = np.random.default_rng(1)
    E = rng.standard_normal((3, 3)); E = 0.5 * (E + E.T)
    u = (X @ E.T).ravel()  # u_a = E x_a
    vol = np.prod(h)
    m = _mandel(E)
    assert abs(u @ K @ u - vol * m @ _D(lam, mu) @ m) < 1e-12 * abs(vol * m @ _D(lam, mu) @ m)


def test_periodic_operator_symmetric_with_translation_nullspace(orc):
    shape = (3, 4, 3)
    rng = np.random.default_rng(2)
    lam = 1.0 + rng.random(shape); mu = 0.5 + rng.random(shape)
    n = np.prod(shape)
    A = np.zeros((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n); e[j] = 1.0
        A[:, j] = orc.el_apply(lam, mu, e.reshape((3,) + shape)).ravel()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    for c in range(3):
        t = np.zeros((3,) + shape); t[c] = 1.0
        assert np.abs(A @ t.ravel()).max() < 1e-13 * np.abs(A).max()
    dg = orc.el_diag(lam, mu).ravel()
    assert np.allclose(dg, np.diag(A), rtol=1e-13, atol=0)


def test_homogeneous_medium_returns_its_stiffness(orc):
    shape = (4, 4, 4)
    lam, mu = np.full(shape, 1.7), np.full(shape, 0.9)
    sols, D = [], _D(1.7, 0.9)
    for j in range(6):
        f = orc.el_rhs(lam, mu, np.eye(6)[j])
        assert np.abs(f).max() < 1e-13
        sols.append(np.zeros((3,) + shape))
    Db = orc.el_effective_stiffness(lam, mu, sols)
    assert np.abs(Db - D).max() < 1e-13


def _solve6(orc, lam, mu, rtol=1e-12):
    sols = []
    for j in range(6):
        u, _ = orc.el_pcg(lam, mu, orc.el_rhs(lam, mu, np.eye(6)[j]), "jacobi", rtol=rtol)
        sols.append(u)
    return orc.el_effective_stiffness(lam, mu, sols), sols


def test_laminate_exact_stiffnesses(orc):
    """Layers normal to x1 (exact piecewise-linear solution): the P-wave
    modulus and the out-of-plane shears are harmonic means, the in-plane
    shear an arithmetic mean."""
    shape = (6, 3, 3)
    E = si.laminate(shape, 0, [1.0, 10.0, 3.0])
    lam, mu = orc.lame(E, 0.3)
    Db, _ = _solve6(orc, lam, mu)
    l1, m1 = lam[:, 0, 0], mu[:, 0, 0]
    assert abs(Db[0, 0] - 1.0 / np.mean(1.0 / (l1 + 2 * m1))) < 1e-9 * Db[0, 0]
    assert abs(Db[3, 3] - 2.0 / np.mean(1.0 / m1)) < 1e-9 * Db[3, 3]
    assert abs(Db[4, 4] - 2.0 / np.mean(1.0 / m1)) < 1e-9 * Db[4, 4]
    assert abs(Db[5, 5] - 2.0 * np.mean(m1)) < 1e-9 * Db[5, 5]


def test_two_phase_bounds_and_symmetry(orc):
    shape = (6, 6, 6)
    ph, _ = si.rsa_inclusions(shape, 1, 2, 0.3, 3)
    E = si.two_phase_kappa(ph, 1.0, 20.0)
    lam, mu = orc.lame(E, 0.3)
    Db, _ = _solve6(orc, lam, mu)
    assert np.abs(Db - Db.T).max() < 1e-8 * np.abs(Db).max()
    Ds = [_D(l, m) for l, m in zip(lam.ravel(), mu.ravel())]
    voigt = np.mean(Ds, axis=0)
    reuss = np.linalg.inv(np.mean([np.linalg.inv(D) for D in Ds], axis=0))
    S = 0.5 * (Db + Db.T)
    assert np.linalg.eigvalsh(voigt - S).min() > -1e-9
    assert np.linalg.eigvalsh(S - reuss).min() > -1e-9


def test_pcg_matches_dense_bordered_solve(orc):
    shape = (3, 3, 3)
    rng = np.random.default_rng(4)
    lam = 1.0 + rng.random(shape); mu = 0.5 + rng.random(shape)
    n = np.prod(shape)
    A = np.zeros((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n); e[j] = 1.0
        A[:, j] = orc.el_apply(lam, mu, e.reshape((3,) + shape)).ravel()
    C = np.zeros((3, 3 * n))
    for c in range(3):
        C[c, c * n:(c + 1) * n] = 1.0
    f = orc.el_rhs(lam, mu, np.array([0.3, -0.1, 0.2, 0.5, 0.0, -0.4])).ravel()
    Kb = np.block([[A, C.T], [C, np.zeros((3, 3))]])
    ref = np.linalg.solve(Kb, np.concatenate([f, np.zeros(3)]))[: 3 * n]
    u, _ = orc.el_pcg(lam, mu, f.reshape((3,) + shape), "jacobi", rtol=1e-13)
    assert np.abs(u.ravel() - ref).max() < 1e-9 * np.abs(ref).max()
