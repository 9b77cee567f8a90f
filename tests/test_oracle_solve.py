"""Pins of the oracle's PCG (Algorithm 1) and effective tensor against the
plain definition of the discrete solution and physics closed forms (no GPU)."""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import synth_inputs as si


def solve_all(orc, kap, kind="jacobi", table=None, rtol=1e-12, max_iter=100000):
    dim = kap.ndim
    loads = [np.eye(dim)[i] for i in range(dim)]
    sols, iters = [], []
    for g in loads:
        f = orc.rhs(kap, g)
        u, it, hist, fr = orc.pcg(kap, f, kind, table=table, rtol=rtol, max_iter=max_iter)
        sols.append(u)
        iters.append(it)
    return loads, sols, iters


@pytest.mark.parametrize("shape", [(8, 8), (8, 8, 8)])
def test_pcg_matches_dense_bordered_solve(orc, shape):
    from oracle import dense
    kap = si.random_field(shape, 21, 0.2, 5.0)
    A = dense.assemble(kap)
    for kind in ("none", "jacobi"):
        for g in np.eye(len(shape)):
            f = orc.rhs(kap, g)
            u_ref = dense.bordered_solve(A, f).reshape(shape)
            u, it, hist, fr = orc.pcg(kap, f, kind, rtol=1e-12)
            assert fr <= 1e-12
            assert np.abs(u - u_ref).max() <= 1e-9 * np.abs(u_ref).max()
            assert abs(u.mean()) < 1e-13


def test_unpreconditioned_pcg_matches_scipy_cg(orc):
    """P = I is textbook CG; compare solutions with scipy's CG on the
    assembled sparse matrix (stopping rules differ: compare solutions)."""
    from oracle import dense
    shape = (10, 9)
    kap = si.random_field(shape, 4, 0.5, 2.0)
    A = scipy.sparse.csr_matrix(dense.assemble(kap))
    f = orc.rhs(kap, [1.0, 0.0])
    x, info = scipy.sparse.linalg.cg(A, f.ravel(), rtol=1e-13, maxiter=5000)
    assert info == 0
    x = x - x.mean()
    u, it, hist, fr = orc.pcg(kap, f, "none", rtol=1e-12)
    assert np.abs(u.ravel() - x).max() <= 1e-9 * np.abs(x).max()


def test_cg_energy_norm_bound(orc):
    """||e_m||_A <= 2 C^m ||e_0||_A with C from cond(D^-1 A) (eq. of Sec. 3.2)
    for Jacobi-CG, checked at every iteration via restarts of max_iter."""
    from oracle import dense
    shape = (8, 8)
    kap = si.random_field(shape, 8, 0.1, 4.0)
    A = dense.assemble(kap)
    f = orc.rhs(kap, [0.3, 1.0])
    u_ref = dense.bordered_solve(A, f)
    D = orc.jacobi_diag(kap).ravel()
    Dm = 1 / np.sqrt(D)
    ev = np.linalg.eigvalsh(Dm[:, None] * A * Dm[None, :])
    cond = ev[-1] / ev[1]  # null space excluded (periodic)
    C = (np.sqrt(cond) - 1) / (np.sqrt(cond) + 1)

    def enorm(e):
        return np.sqrt(e @ A @ e)

    e0 = enorm(u_ref)
    for m in range(1, 30, 3):
        u, it, hist, fr = orc.pcg(kap, f, "jacobi", rtol=0.0, max_iter=m)
        assert it == m
        assert enorm(u.ravel() - u_ref) <= 2 * C ** m * e0 * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_returns_own_conductivity(orc, dim):
    """The rhs vanishes (up to rounding), so the discrete fluctuation is 0
    and the flux average returns kappa I."""
    kap = np.full((6,) * dim, 3.7)
    loads = [np.eye(dim)[i] for i in range(dim)]
    for g in loads:
        assert np.abs(orc.rhs(kap, g)).max() < 1e-15
    sols = [np.zeros_like(kap) for _ in loads]
    kb = orc.effective_tensor(kap, sols, loads)
    assert np.allclose(kb, 3.7 * np.eye(dim), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dim,axis", [(2, 0), (2, 1), (3, 0), (3, 2)])
def test_laminate_harmonic_and_arithmetic_means(orc, dim, axis):
    """Voxel-aligned layers normal to x_axis: the exact solution is piecewise
    linear along x_axis and lies in the FE space, so kappa_bar is exactly the
    harmonic mean normal to the layers and the arithmetic mean along them."""
    shape = (8,) * dim
    vals = [1.0, 10.0, 3.0]
    kap = si.laminate(shape, axis, vals, seed=17)
    layer = kap.reshape(-1)[:0]  # noqa: F841
    prof = np.moveaxis(kap, axis, 0)[(slice(None),) + (0,) * (dim - 1)]
    harm = 1.0 / np.mean(1.0 / prof)
    arit = np.mean(prof)
    loads, sols, iters = solve_all(orc, kap)
    kb = orc.effective_tensor(kap, sols, loads)
    expect = np.eye(dim) * arit
    expect[axis, axis] = harm
    assert np.allclose(kb, expect, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("shape", [(16, 16), (8, 8, 8)])
def test_two_phase_bounds_symmetry_energy(orc, shape):
    """Voigt/Reuss bounds, symmetry, and flux form = energy form at the
    discrete solution (Galerkin orthogonality)."""
    ph, _ = si.rsa_inclusions(shape, 2, 3, 0.3, 9)
    kap = si.two_phase_kappa(ph, 1.0, 10.0)
    loads, sols, iters = solve_all(orc, kap)
    kb = orc.effective_tensor(kap, sols, loads)
    ke = orc.energy_tensor(kap, sols, loads)
    assert np.abs(kb - kb.T).max() <= 1e-9 * np.abs(kb).max()
    assert np.abs(kb - ke).max() <= 1e-9 * np.abs(kb).max()
    ev = np.linalg.eigvalsh(0.5 * (kb + kb.T))
    voigt = kap.mean()
    reuss = 1.0 / np.mean(1.0 / kap)
    assert reuss - 1e-12 <= ev[0] and ev[-1] <= voigt + 1e-12


def test_iteration_count_is_loop_passes(orc):
    shape = (8, 8)
    kap = si.random_field(shape, 1, 0.5, 1.5)
    f = orc.rhs(kap, [1.0, 0.0])
    u, it, hist, fr = orc.pcg(kap, f, "jacobi", rtol=1e-6)
    assert len(hist) == it + 1
    assert hist[-1] <= 1e-6 * hist[0] and hist[-2] > 1e-6 * hist[0]
    assert hist[0] == pytest.approx(np.abs(f).max())
