"""Pins of the oracle's unitary transform, UNO preconditioner and FANS table
(Sec. 3.3.4, Sec. 4.2) against library routines, closed forms, the spectrum
lemma and the values Table 2 prints for FANS (no GPU)."""
import json
import os

import numpy as np
import pytest

import synth_inputs as si

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table2.json")))


@pytest.mark.parametrize("shape", [(8, 8), (12, 10), (7, 5), (6, 5, 4), (9, 3, 8), (30, 4)])
def test_fft_matches_numpy_and_dft(orc, shape):
    x = si.random_field(shape, 3) + 1j * si.random_field(shape, 4)
    X = orc.fft(x)
    assert np.abs(X - np.fft.fftn(x, norm="ortho")).max() < 1e-13 * np.abs(X).max()
    assert np.abs(orc.fft(X, inverse=True) - x).max() < 1e-13
    # Parseval (unitary) and impulse -> constant 1/sqrt(n)
    assert np.linalg.norm(X) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    e = np.zeros(shape)
    e[(0,) * len(shape)] = 1.0
    assert np.allclose(orc.fft(e), 1.0 / np.sqrt(np.prod(shape)), atol=1e-15)


def test_fft_brute_force_dft_1d_like(orc):
    n = 15
    x = si.random_field((n, 1), 5)[:, 0] + 0j
    W = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) / np.sqrt(n)
    got = orc.fft(x.reshape(n, 1))[:, 0]  # length-1 second axis: identity
    assert np.abs(got - W @ x).max() < 1e-13


@pytest.mark.parametrize("dim,M", [(2, 0), (2, 3), (3, 1), (3, 2)])
def test_num_weights_matches_mode_table(orc, dim, M):
    """N_w = C (k_max + 1) with k_max = (2M+1)^(d-1)(M+1) - 1 for periodic BC."""
    assert orc.num_weights(dim, M) == (2 * M + 1) ** (dim - 1) * (M + 1)


@pytest.mark.parametrize("shape", [(8, 8), (6, 6, 6)])
def test_constant_table_is_scaled_projection(orc, shape):
    """Phi = c on every mode except 0: P r = c (r - mean r)."""
    r = si.random_field(shape, 1)
    tab = np.full(shape, 2.5)
    tab[(0,) * len(shape)] = 0.0
    s = orc.table_apply(tab, r)
    assert np.abs(s - 2.5 * (r - r.mean())).max() < 1e-13
    # UNO with theta = (c, 0, ..., 0) is the same map (bypass only)
    M = 2
    th = np.zeros(orc.num_weights(len(shape), M))
    th[0] = np.sqrt(2.5)
    assert np.abs(orc.uno_apply(th, M, r) - s).max() < 1e-13


@pytest.mark.parametrize("shape", [(8, 8), (10, 6), (6, 6, 6)])
def test_fans_table_inverts_reference_operator(orc, shape):
    """FANS: A_ref P_F r = r - mean(r) (the pseudo-inverse on the periodic grid)."""
    r = si.random_field(shape, 2)
    tab = orc.fans_table(0.6, shape)
    s = orc.table_apply(tab, r)
    back = orc.fe_apply(np.full(shape, 0.6), s)
    assert np.abs(back - (r - r.mean())).max() < 1e-12 * np.abs(r).max()


def test_fans_spectrum_matches_table2(orc):
    """Two-phase kappa in {1, 0.2}, kappa_ref = arithmetic mean 0.6: the
    spectrum of P_F A on the complement of the constants is [1/3, 5/3] with
    condition number 5 (Table 2 prints 0.3333, 1.6667, 5.0000)."""
    from oracle import dense
    shape = (12, 12)
    ph, _ = si.rsa_inclusions(shape, 2, 3, 0.4, 5)
    kap = si.two_phase_kappa(ph, *GOLD["kappa_phases"])
    A = dense.assemble(kap)
    tab = orc.fans_table(0.6, shape)
    P = dense.operator_matrix(lambda v: orc.table_apply(tab, v), shape)
    ev = np.sort(np.linalg.eigvals(P @ A).real)
    assert abs(ev[0]) < 1e-12
    lo, hi = ev[1], ev[-1]
    row = GOLD["rows"]["FANS"]
    assert round(lo, 4) == row["lambda_min"]
    assert round(hi, 4) == row["lambda_max"]
    assert round(hi / lo, 4) == row["cond"]


def test_fans_cg_iterations_within_bound(orc):
    """FANS-CG for R = 5 reaches 1e-6 within the CG estimate of Table 2
    (15 passes; the paper's sample took 14)."""
    shape = (32, 32)
    ph, _ = si.rsa_inclusions(shape, 3, 5, 0.3, 2)
    kap = si.two_phase_kappa(ph, *GOLD["kappa_phases"])
    tab = orc.fans_table(0.6, shape)
    f = orc.rhs(kap, [1.0, 0.0])
    u, it, hist, fr = orc.pcg(kap, f, "table", table=tab, rtol=1e-6)
    assert it <= GOLD["rows"]["FANS"]["n_iter_est"] + 1


@pytest.mark.parametrize("shape,M", [((8, 8), 2), ((7, 9), 3), ((6, 5, 5), 2), ((6, 6, 4), 1)])
def test_uno_spectrum_lemma_symmetry_realness(orc, shape, M):
    """Spectrum lemma (Sec. 4.2.3): eig(P) = union of table values; P is
    symmetric; the output is real."""
    from oracle import dense
    th = si.random_theta(orc.num_weights(len(shape), M), 7)
    tab = orc.uno_table(shape, M, th)
    P = dense.operator_matrix(lambda v: orc.uno_apply(th, M, v), shape)
    assert np.abs(P - P.T).max() < 1e-13 * np.abs(P).max()
    assert np.abs(np.sort(np.linalg.eigvalsh(P)) - np.sort(tab.ravel())).max() < 1e-12 * tab.max()
    s, im = orc.table_apply(tab, si.random_field(shape, 3), return_imag=True)
    assert im < 1e-13 * np.abs(s).max()


def test_uno_table_structure(orc):
    """Modes outside the learned block carry only the bypass theta0^2; a
    learned mode k with k_d > 0 and its reflection -k carry theta0^2 +
    theta_i^2; the zero mode carries 0."""
    shape, M = (9, 9, 8), 2
    nw = orc.num_weights(3, M)
    th = si.random_theta(nw, 4)
    tab = orc.uno_table(shape, M, th)
    W = th[0] ** 2
    assert tab[0, 0, 0] == 0.0
    assert tab[4, 4, 4] == pytest.approx(W)          # far mode, bypass only
    # k = (1, -2, 1): lexicographic slot over (k1+M, k2+M, k3), zero skipped
    L = ((1 + M) * (2 * M + 1) + (-2 + M)) * (M + 1) + 1
    L0 = (M * (2 * M + 1) + M) * (M + 1)
    slot = L + 1 if L < L0 else L
    assert tab[1, 9 - 2, 1] == pytest.approx(W + th[slot] ** 2)
    assert tab[9 - 1, 2, 8 - 1] == pytest.approx(W + th[slot] ** 2)  # -k


def test_impulse_response_is_learned_greens_function(orc):
    """P applied to a unit impulse is the inverse transform of the table, i.e.
    the learned fundamental solution (Sec. 6.3), shifted to the impulse."""
    shape, M = (8, 8), 2
    th = si.random_theta(orc.num_weights(2, M), 11)
    tab = orc.uno_table(shape, M, th)
    e = np.zeros(shape)
    e[3, 5] = 1.0
    g = orc.uno_apply(th, M, e)
    G = np.real(np.fft.ifftn(tab)) * 1.0  # kernel of the circulant map
    assert np.abs(g - np.roll(G, (3, 5), axis=(0, 1))).max() < 1e-13
