"""GPU: gradient of the effective conductivity with respect to every voxel
conductivity (hand-written energy-density kernel; the cell problem is
self-adjoint) against the oracle's Gauss-quadrature gradient, Euler's
identity and central differences at the 64^3 benchmark size, and the
autograd wrapper."""
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


def _kappa(shape, seed, contrast=100.0):
    ph, _ = si.rsa_inclusions(shape, 1 if min(shape) < 10 else 2, 2 if min(shape) < 10 else 4, 0.3, seed)
    return si.two_phase_kappa(ph, 1.0, contrast)


def _oracle_solutions(orc, kap, loads):
    return [orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-13)[0] for g in loads]


@pytest.mark.parametrize("shape", [(8, 8), (5, 7), (6, 5, 4), (12, 10, 8), (1, 6, 4)])
def test_gradient_kernel_matches_oracle(orc, uno, shape):
    """Same fields in (the oracle's solutions), same densities out."""
    dim = len(shape)
    kap = _kappa(shape, 51, 10.0)
    rng = np.random.default_rng(52)
    loads = np.eye(dim) + 0.3 * rng.standard_normal((dim, dim))  # a general invertible load set
    sols = _oracle_solutions(orc, kap, list(loads))
    ref = orc.kbar_grad(kap, sols, list(loads))
    got = uno.effective_tensor_grad(shape, loads, T(np.stack(sols))).cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-12 * scale
    w = rng.standard_normal((dim, dim))
    vjp = uno.effective_tensor_grad(shape, loads, T(np.stack(sols)), weights=w).cpu().numpy()
    assert np.abs(vjp - np.einsum("ij,ij...->...", w, ref)).max() < 1e-12 * scale * np.abs(w).sum()


@pytest.mark.parametrize("shape", [(16, 16), (12, 10, 14)])
def test_solve_and_gradient_match_oracle(orc, uno, shape):
    dim = len(shape)
    kap = _kappa(shape, 53)
    loads = np.eye(dim)
    u, infos = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="jacobi", rtol=1e-12)
    assert all(i["converged"] for i in infos)
    got = uno.effective_tensor_grad(shape, loads, u).cpu().numpy()
    ref = orc.kbar_grad(kap, _oracle_solutions(orc, kap, list(loads)), list(loads))
    assert np.abs(got - ref).max() < 1e-8 * np.abs(ref).max()


def test_gradient_64cubed_euler_and_central_differences(uno):
    """The differentiation workload: 64^3 spheres at contrast 100, gradient of
    kappa_bar w.r.t. all 262144 voxel conductivities; Euler's identity over
    all voxels and central differences (GPU solves) on 32 random voxels."""
    cfg = dict(si.CONFIG_3D_64)
    kapn = si.microstructure(cfg, 1000)[0]
    kap = T(kapn)
    shape = kapn.shape
    loads = np.eye(3)
    kw = dict(kind="jacobi", rtol=1e-12, max_iter=50000)
    u, infos = uno.pcg_solve_batch(kap, macro_loads=loads, **kw)
    kb = uno.effective_tensor(kap, loads, u)
    grad = uno.effective_tensor_grad(shape, loads, u)
    euler = torch.einsum("ijxyz,xyz->ij", grad, kap).cpu().numpy()
    assert np.abs(euler - kb).max() < 1e-8 * np.abs(kb).max()
    gs = grad.cpu().numpy()
    rng = np.random.default_rng(54)
    worst = 0.0
    for _ in range(32):
        e = tuple(int(rng.integers(0, s)) for s in shape)
        h = 1e-2 * kapn[e]
        kbs = []
        for sgn in (1.0, -1.0):
            kp = kap.clone()
            kp[e] += sgn * h
            up, _ = uno.pcg_solve_batch(kp, macro_loads=loads, **kw)
            kbs.append(uno.effective_tensor(kp, loads, up))
        fd = (kbs[0] - kbs[1]) / (2 * h)
        an = gs[(slice(None), slice(None)) + e]
        worst = max(worst, np.abs(fd - an).max() / np.abs(an).max())
    print("64^3 central differences vs gradient: worst rel %.2e" % worst, flush=True)
    assert worst < 2e-3


def test_autograd_function(uno):
    shape = (12, 10, 8)
    kap = T(_kappa(shape, 55)).requires_grad_(True)
    kb = uno.EffectiveConductivity.apply(kap, "jacobi", None, 1e-12)
    w = torch.tensor([[1.0, 0.5, 0.0], [0.5, 2.0, -1.0], [0.0, -1.0, 0.3]], dtype=torch.float64, device=DEV)
    (kb * w).sum().backward()
    loads = np.eye(3)
    u, _ = uno.pcg_solve_batch(kap.detach(), macro_loads=loads, kind="jacobi", rtol=1e-12)
    full = uno.effective_tensor_grad(shape, loads, u)
    ref = torch.einsum("ij,ij...->...", w, full)
    assert torch.allclose(kap.grad, ref, rtol=1e-9, atol=1e-14)
    # Euler: sum_e kappa_e d(w:kbar)/d kappa_e = w : kbar
    assert abs(float((kap.grad * kap.detach()).sum()) - float((kb.detach() * w).sum())) < 1e-8 * float(kb.detach().abs().max())
