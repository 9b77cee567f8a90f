"""Pins of the oracle's finite-element operator, rhs and Jacobi diagonal
against closed forms and values the paper prints (no GPU)."""
import json
import os

import numpy as np
import pytest

import synth_inputs as si

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table2.json")))


def hom_symbol(shape, L0=1.0):
    """Closed-form eigenvalues of the unit-conductivity periodic operator on
    cubic voxels, derived by hand from the bilinear/trilinear element:
    2D: (2/3)(4 - c1 - c2 - 2 c1 c2); 3D: (2h/3)(4 - (c1c2 + c1c3 + c2c3) - c1c2c3),
    c_i = cos(2 pi k_i / N_i)."""
    cs = np.meshgrid(*[np.cos(2 * np.pi * np.arange(n) / n) for n in shape], indexing="ij")
    if len(shape) == 2:
        c1, c2 = cs
        return (2.0 / 3.0) * (4 - c1 - c2 - 2 * c1 * c2)
    c1, c2, c3 = cs
    h = L0 / shape[0]
    return (2 * h / 3.0) * (4 - (c1 * c2 + c1 * c3 + c2 * c3) - c1 * c2 * c3)


@pytest.mark.parametrize("shape", [(6, 6), (5, 7), (6, 6, 6), (4, 5, 3)])
def test_operator_symmetric_and_constant_nullspace(orc, shape):
    from oracle import dense
    kap = si.random_field(shape, 11, 0.1, 3.0)
    A = dense.assemble(kap)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(A @ np.ones(A.shape[0])).max() <= 1e-13 * np.abs(A).max()
    # positive semidefinite with a one-dimensional null space (periodic BC, Sec. 4.2 remark)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 and ev[1] > 1e-8


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (6, 6, 6), (4, 4, 4)])
def test_homogeneous_spectrum_matches_symbol(orc, shape):
    from oracle import dense
    if len(shape) == 3 and len(set(shape)) > 1:
        pytest.skip("closed form written for cubic voxels")
    if len(shape) == 2 and len(set(shape)) > 1:
        # rectangular pixels: compare against eigenvalues computed by the DFT
        kap = np.ones(shape)
        A = dense.assemble(kap)
        T = orc.fans_table(1.0, shape)
        lam = np.where(T != 0, 1.0 / np.where(T != 0, T, 1), 0.0)
        assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam.ravel()), atol=1e-12)
        return
    A = dense.assemble(np.ones(shape))
    ev = np.sort(np.linalg.eigvalsh(A))
    assert np.abs(ev - np.sort(hom_symbol(shape).ravel())).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_max_is_4_kappa_h_pow_dminus2(orc, dim):
    """Homogeneous largest eigenvalue 4 kappa h^(d-2): the paper prints
    3.9998 for kappa_max = 1 in 2D (Table 2, CG row)."""
    from oracle import dense
    shape = (8,) * dim
    kap = np.full(shape, 2.5)
    ev = np.linalg.eigvalsh(dense.assemble(kap))
    h = 1.0 / 8
    assert ev[-1] == pytest.approx(4 * 2.5 * h ** (dim - 2), rel=1e-13)


def test_lambda_max_two_phase_2d_matches_table2(orc):
    """Two-phase 2D sample with kappa in {1, 0.2}: lambda_max(A) is bounded
    by 4 kappa_max (A <= kappa_max A(1) element by element) and approaches it
    as the largest kappa = 1 region grows (paper, 400^2: 3.9998); and
    lambda_max(D^-1 A) = 1.5 (paper: 1.5000)."""
    from oracle import dense
    ph, _ = si.rsa_inclusions((32, 32), 3, 5, 0.3, 3)
    kap = si.two_phase_kappa(ph, *GOLD["kappa_phases"])
    A = dense.assemble(kap)
    lmax = np.linalg.eigvalsh(A)[-1]
    assert 3.95 < lmax <= 4.0 + 1e-12
    assert round(lmax, 1) == round(GOLD["rows"]["CG"]["lambda_max"], 1)
    D = orc.jacobi_diag(kap).ravel()
    Dm = 1.0 / np.sqrt(D)
    ljac = np.linalg.eigvalsh(Dm[:, None] * A * Dm[None, :])[-1]
    assert round(ljac, 4) == GOLD["rows"]["Jac-CG"]["lambda_max"]


@pytest.mark.parametrize("dim", [2, 3])
def test_jacobi_diagonal_closed_form(orc, dim):
    """diag A = (8/3) kappa in 2D and (8h/3) kappa in 3D for homogeneous kappa
    (self-coupling of the bilinear/trilinear element times 2^d voxels)."""
    shape = (6,) * dim
    d = orc.jacobi_diag(np.full(shape, 3.0))
    h = 1.0 / 6
    expect = 3.0 * (8.0 / 3.0) * (h if dim == 3 else 1.0)
    assert np.allclose(d, expect, rtol=1e-14)
    from oracle import dense
    kap = si.random_field(shape, 2, 0.5, 2.0)
    assert np.allclose(orc.jacobi_diag(kap).ravel(), np.diag(dense.assemble(kap)), rtol=1e-13)


@pytest.mark.parametrize("shape", [(1, 5, 3), (2, 4, 3), (1, 6), (5, 1, 1)])
def test_jacobi_diagonal_is_assembled_diagonal_on_thin_grids(orc, shape):
    """P_Jac = 1 / A_ii of the assembled matrix (Sec. 3.2), also where an
    axis has one or two voxels and element nodes coincide."""
    from oracle import dense
    kap = si.random_field(shape, 12, 0.5, 2.0)
    assert np.allclose(orc.jacobi_diag(kap).ravel(), np.diag(dense.assemble(kap)), rtol=1e-13)


@pytest.mark.parametrize("shape", [(8, 8), (6, 5, 4)])
def test_rhs_invariants(orc, shape):
    """Sum f = 0 (f lies in the range of the periodic operator) and f = 0 for
    a homogeneous material (Sec. 5.1 decomposition)."""
    dim = len(shape)
    g = np.linspace(0.3, 1.1, dim)
    kap = si.random_field(shape, 5, 0.1, 10.0)
    f = orc.rhs(kap, g)
    assert abs(f.sum()) < 1e-12 * np.abs(f).max()
    assert np.abs(orc.rhs(np.full(shape, 7.0), g)).max() < 1e-12


def test_rhs_vanishes_for_load_along_layers(orc):
    """For a laminate whose conductivity varies only along x1 and a load
    along x2, div(kappa gbar) = 0, so the discrete rhs vanishes."""
    kap = si.laminate((8, 8), 0, [1.0, 10.0])
    f = orc.rhs(kap, [0.0, 1.0])
    assert np.abs(f).max() < 1e-13
