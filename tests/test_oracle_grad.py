"""Pins of the oracle's gradient of the effective conductivity with respect
to the voxel conductivities (self-adjoint cell problem: the derivative is
the element energy density of the forward solutions).  Each pin fixes it by
something other than its own formula: central finite differences of the
oracle's solve + effective tensor, Euler's identity for the degree-1
homogeneous map kappa -> kappa_bar, the homogeneous medium, and the
closed-form laminate means."""
import numpy as np
import pytest

import synth_inputs as si


def _solve_all(orc, kap, loads, rtol=1e-13):
    return [orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=rtol)[0] for g in loads]


def _kbar(orc, kap, loads):
    return orc.effective_tensor(kap, _solve_all(orc, kap, loads), loads)


@pytest.mark.parametrize("shape,nvox", [((6, 6), None), ((4, 4, 4), 6)])
def test_gradient_matches_central_differences(orc, shape, nvox):
    ph, _ = si.rsa_inclusions(shape, 1, 2, 0.3, 3)
    kap = si.two_phase_kappa(ph, 1.0, 5.0) * (1.0 + 0.2 * si.random_field(shape, 4))
    loads = list(np.eye(len(shape)))
    grad = orc.kbar_grad(kap, _solve_all(orc, kap, loads), loads)
    rng = np.random.default_rng(5)
    idx = list(np.ndindex(shape)) if nvox is None else [tuple(rng.integers(0, s) for s in shape) for _ in range(nvox)]
    scale = np.abs(grad).max()
    for e in idx:
        h = 1e-4 * kap[e]
        kp, km = kap.copy(), kap.copy()
        kp[e] += h
        km[e] -= h
        fd = (_kbar(orc, kp, loads) - _kbar(orc, km, loads)) / (2 * h)
        assert np.abs(fd - grad[(slice(None), slice(None)) + e]).max() < 1e-6 * scale, e


@pytest.mark.parametrize("shape", [(8, 8), (6, 5, 4)])
def test_euler_identity(orc, shape):
    """kappa_bar(t kappa) = t kappa_bar(kappa), so sum_e kappa_e d kappa_bar /
    d kappa_e = kappa_bar."""
    ph, _ = si.rsa_inclusions(shape, 1, 2, 0.3, 6)
    kap = si.two_phase_kappa(ph, 1.0, 20.0)
    loads = list(np.eye(len(shape)))
    sols = _solve_all(orc, kap, loads)
    kb = orc.effective_tensor(kap, sols, loads)
    grad = orc.kbar_grad(kap, sols, loads)
    euler = np.tensordot(grad, kap, axes=len(shape))
    assert np.abs(euler - kb).max() < 1e-10 * np.abs(kb).max()
    assert np.abs(grad - np.swapaxes(grad, 0, 1)).max() < 1e-13 * np.abs(grad).max()


def test_homogeneous_medium(orc):
    """theta = 0: every voxel contributes delta_ij / N_e."""
    shape = (4, 5, 3)
    kap = np.full(shape, 2.5)
    loads = list(np.eye(3))
    grad = orc.kbar_grad(kap, [np.zeros(shape)] * 3, loads)
    ne = np.prod(shape)
    for i in range(3):
        for j in range(3):
            assert np.allclose(grad[i, j], (i == j) / ne, rtol=0, atol=1e-15)


def test_laminate_layer_sums(orc):
    """Layers normal to x1: kappa_bar_11 is the harmonic mean over layers,
    kappa_bar_22 the arithmetic one; summing the voxel derivatives over a
    layer gives the derivatives of these means with respect to the layer."""
    shape = (6, 4, 4)
    vals = [1.0, 4.0, 2.0]
    kap = si.laminate(shape, 0, vals)
    loads = list(np.eye(3))
    sols = _solve_all(orc, kap, loads)
    grad = orc.kbar_grad(kap, sols, loads)
    nl = shape[0]
    kl = kap[:, 0, 0]
    k11 = 1.0 / np.mean(1.0 / kl)
    for L in range(nl):
        s11 = grad[0, 0, L].sum()
        s22 = grad[1, 1, L].sum()
        assert abs(s11 - k11 ** 2 / (nl * kl[L] ** 2)) < 1e-11
        assert abs(s22 - 1.0 / nl) < 1e-11
