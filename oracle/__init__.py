"""FP64 CPU oracle for UNO-CG (arXiv 2508.02681).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package,
which shares no code with it.

Thin numpy/ctypes wrapper around ``oracle.c`` (built with gcc on first use or
by ``build()``), plus dense reference helpers in :mod:`oracle.dense`.
Every routine cites the passage of the paper it follows in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, single thread)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    i32, f64 = ctypes.c_int32, ctypes.c_double
    lib.orc_element_matrix.argtypes = [i32, _ip, _dp, _dp]
    lib.orc_fe_apply.argtypes = [i32, _ip, _dp, _dp, _dp, _dp]
    lib.orc_jacobi_diag.argtypes = [i32, _ip, _dp, _dp, _dp]
    lib.orc_rhs.argtypes = [i32, _ip, _dp, _dp, _dp, _dp]
    lib.orc_flux_average.argtypes = [i32, _ip, _dp, _dp, _dp, _dp, _dp]
    lib.orc_energy_average.argtypes = [i32, _ip, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_energy_average.restype = f64
    lib.orc_energy_density.argtypes = [i32, _ip, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_fft_nd.argtypes = [i32, _ip, _dp, i32]
    lib.orc_el_element_matrix.argtypes = [_ip, _dp, f64, f64, _dp]
    lib.orc_el_apply.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    lib.orc_el_diag.argtypes = [_ip, _dp, _dp, _dp, _dp]
    lib.orc_el_rhs.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    lib.orc_el_stress_average.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_el_pcg.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, i32, _dp, f64, i32]
    lib.orc_psi3.argtypes = [_dp, _dp]
    lib.orc_uno3_table.argtypes = [_ip, i32, _dp, _dp]
    lib.orc_uno3_apply.argtypes = [_ip, _dp, _dp, _dp]
    lib.orc_uno3_apply.restype = f64
    lib.orc_train3_features.argtypes = [_ip, i32, _dp, _dp, _dp, _dp, _dp]
    lib.orc_train3_loss.argtypes = [_ip, i32, _dp, _dp, _dp, f64]
    lib.orc_train3_loss.restype = f64
    lib.orc_train3_grad_hess.argtypes = [_ip, i32, _dp, _dp, _dp, _dp, _dp]
    lib.orc_el_pcg.restype = i32
    lib.orc_uno_num_weights.argtypes = [i32, i32]
    lib.orc_uno_num_weights.restype = ctypes.c_int64
    lib.orc_uno_table.argtypes = [i32, _ip, i32, _dp, _dp]
    lib.orc_table_apply.argtypes = [i32, _ip, _dp, _dp, _dp]
    lib.orc_table_apply.restype = f64
    lib.orc_fans_table.argtypes = [i32, _ip, _dp, f64, _dp]
    lib.orc_pcg.argtypes = [i32, _ip, _dp, _dp, _dp, _dp, i32, _dp, f64, i32, _dp, _dp]
    lib.orc_pcg.restype = i32
    lib.orc_train_features.argtypes = [i32, _ip, i32, _dp, _dp, _dp, _dp, _dp]
    lib.orc_train_loss.argtypes = [i32, _ip, i32, _dp, _dp, _dp, f64]
    lib.orc_train_loss.restype = f64
    lib.orc_train_closed_form.argtypes = [i32, _ip, i32, _dp, _dp, _dp]
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _shape_args(shape, L0=1.0, h=None):
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    n = np.array(list(shape) + [1] * (3 - dim), dtype=np.int32)
    if h is None:
        h = [L0 / s for s in shape]  # domain [-L0/2, L0/2]^d (Sec. 5)
    hh = np.array(list(h) + [1.0] * (3 - dim), dtype=np.float64)
    return dim, n, hh


def element_matrix(shape, L0=1.0, h=None) -> np.ndarray:
    """Unit-conductivity element stiffness (2^d x 2^d), Gauss-integrated."""
    lib = _load()
    dim, n, hh = _shape_args(shape, L0, h)
    K = np.zeros((1 << dim) ** 2)
    lib.orc_element_matrix(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(K))
    return K.reshape(1 << dim, 1 << dim)


def fe_apply(kappa, u, L0=1.0, h=None) -> np.ndarray:
    """y = A(kappa) u by the element loop."""
    lib = _load()
    kappa = _f64(kappa)
    u = _f64(u)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    y = np.empty_like(u)
    lib.orc_fe_apply(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), _ptr(u), _ptr(y))
    return y


def jacobi_diag(kappa, L0=1.0, h=None) -> np.ndarray:
    lib = _load()
    kappa = _f64(kappa)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    d = np.empty_like(kappa)
    lib.orc_jacobi_diag(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), _ptr(d))
    return d


def rhs(kappa, gbar, L0=1.0, h=None) -> np.ndarray:
    lib = _load()
    kappa = _f64(kappa)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    g = _f64(gbar)
    f = np.empty_like(kappa)
    lib.orc_rhs(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), _ptr(g), _ptr(f))
    return f


def flux_average(kappa, gbar, theta, L0=1.0, h=None) -> np.ndarray:
    lib = _load()
    kappa = _f64(kappa)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    g = _f64(gbar)
    t = _f64(theta)
    out = np.zeros(dim)
    lib.orc_flux_average(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), _ptr(g), _ptr(t), _ptr(out))
    return out


def energy_average(kappa, g1, t1, g2, t2, L0=1.0, h=None) -> float:
    lib = _load()
    kappa = _f64(kappa)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    a = [_f64(x) for x in (g1, t1, g2, t2)]
    return lib.orc_energy_average(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), *[_ptr(x) for x in a])


def fft(x, inverse=False) -> np.ndarray:
    """Unitary d-dimensional DFT (own recursive mixed-radix code)."""
    lib = _load()
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    dim, n, _ = _shape_args(a.shape)
    lib.orc_fft_nd(dim, n.ctypes.data_as(_ip), a.ctypes.data_as(_dp), 1 if inverse else -1)
    return a


def num_weights(dim: int, M: int) -> int:
    """Length of theta = 1 + k_max = (2M+1)^(d-1) (M+1)."""
    return int(_load().orc_uno_num_weights(dim, M))


def check_modes(shape, M):
    if M < 0 or any(2 * M + 1 > s for s in shape):
        raise ValueError("need 0 <= M and 2M+1 <= N_i on every axis")


def uno_table(shape, M, theta) -> np.ndarray:
    """Full-spectrum preconditioner table Phi(k) (symmetrized, Phi(0)=0)."""
    lib = _load()
    check_modes(shape, M)
    dim, n, _ = _shape_args(shape)
    theta = _f64(theta)
    if theta.size != num_weights(dim, M):
        raise ValueError("theta has %d entries, expected %d" % (theta.size, num_weights(dim, M)))
    tab = np.empty(tuple(shape))
    lib.orc_uno_table(dim, n.ctypes.data_as(_ip), int(M), _ptr(theta), _ptr(tab))
    return tab


def fans_table(kappa_ref, shape, L0=1.0, h=None) -> np.ndarray:
    lib = _load()
    dim, n, hh = _shape_args(shape, L0, h)
    tab = np.empty(tuple(shape))
    lib.orc_fans_table(dim, n.ctypes.data_as(_ip), _ptr(hh), float(kappa_ref), _ptr(tab))
    return tab


def table_apply(table, r, return_imag=False):
    """s = T^H diag(table) T r."""
    lib = _load()
    table = _f64(table)
    r = _f64(r)
    dim, n, _ = _shape_args(r.shape)
    s = np.empty_like(r)
    im = lib.orc_table_apply(dim, n.ctypes.data_as(_ip), _ptr(table), _ptr(r), _ptr(s))
    return (s, im) if return_imag else s


def uno_apply(theta, M, r):
    return table_apply(uno_table(r.shape, M, theta), r)


KIND = {"none": 0, "jacobi": 1, "table": 2, "uno": 2, "fans": 2}


def pcg(kappa, f, kind="jacobi", table=None, rtol=1e-6, max_iter=100000, u0=None, L0=1.0, h=None):
    """Algorithm 1; returns (u, iters, res_hist, final_rel)."""
    lib = _load()
    kappa = _f64(kappa)
    f = _f64(f)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    u = np.zeros_like(f) if u0 is None else _f64(u0).copy()
    k = KIND[kind]
    tab = _f64(table) if k == 2 else np.zeros(1)
    hist = np.zeros(max_iter + 1)
    fr = ctypes.c_double(0.0)
    it = lib.orc_pcg(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(kappa), _ptr(f), _ptr(u), k, _ptr(tab),
                     float(rtol), int(max_iter), _ptr(hist), ctypes.byref(fr))
    return u, int(it), hist[: it + 1].copy(), fr.value


def timed_pcg(job):
    """(passes, seconds) of one pcg(kappa, rhs(kappa, gbar), kind, table of
    (M, theta) for kind "uno", rtol) call; job = (kappa, gbar, kind, theta, M,
    rtol).  For timing the oracle in worker processes."""
    import time
    kappa, gbar, kind, theta, M, rtol = job
    table = uno_table(kappa.shape, M, theta) if kind == "uno" else None
    f = rhs(kappa, gbar)
    t = time.perf_counter()
    _, it, _, _ = pcg(kappa, f, kind, table=table, rtol=rtol)
    return it, time.perf_counter() - t


def pcg_solution(job):
    """The solution u of the same call as timed_pcg (for worker processes)."""
    kappa, gbar, kind, theta, M, rtol = job
    table = uno_table(kappa.shape, M, theta) if kind == "uno" else None
    return pcg(kappa, rhs(kappa, gbar), kind, table=table, rtol=rtol)[0]


def effective_tensor(kappa, solutions, loads, L0=1.0, h=None) -> np.ndarray:
    """kappa_bar from flux averages: column j = <kappa (g_j + grad theta_j)>,
    then kappa_bar = F G^{-1} for the load matrix G = [g_1 ... g_d]."""
    kappa = _f64(kappa)
    G = np.array(loads, dtype=np.float64).T
    F = np.stack([flux_average(kappa, g, t, L0, h) for g, t in zip(loads, solutions)], axis=1)
    return F @ np.linalg.inv(G)


def energy_tensor(kappa, solutions, loads, L0=1.0, h=None) -> np.ndarray:
    d = len(loads)
    E = np.zeros((d, d))
    for i in range(d):
        for j in range(d):
            E[i, j] = energy_average(kappa, loads[i], solutions[i], loads[j], solutions[j], L0, h)
    G = np.array(loads, dtype=np.float64).T
    Gi = np.linalg.inv(G)
    return Gi.T @ E @ Gi


def kbar_grad(kappa, solutions, loads, L0=1.0, h=None) -> np.ndarray:
    """d kappa_bar_ij / d kappa_e for every voxel e (array d x d x grid): the
    element energy densities D_ab(e) of the load pairs (exact total
    derivatives of g_a . kappa_bar g_b at the discrete solutions), mapped
    through kappa_bar = G^-T E G^-1 for the load matrix G = [g_1 ... g_d]."""
    lib = _load()
    kappa = _f64(kappa)
    dim, n, hh = _shape_args(kappa.shape, L0, h)
    d = len(loads)
    D = np.zeros((d, d) + kappa.shape)
    for a in range(d):
        for b in range(a, d):
            out = np.zeros(kappa.shape)
            lib.orc_energy_density(dim, n.ctypes.data_as(_ip), _ptr(hh), _ptr(_f64(loads[a])), _ptr(_f64(solutions[a])),
                                   _ptr(_f64(loads[b])), _ptr(_f64(solutions[b])), _ptr(out))
            D[a, b] = out
            D[b, a] = out
    Gi = np.linalg.inv(np.array(loads, dtype=np.float64).T)
    return np.einsum("ai,ab...,bj->ij...", Gi, D, Gi)


def train_features(f_list, u_list):
    """(alpha, beta, delta) over the full Fourier grid."""
    lib = _load()
    f = _f64(np.stack(f_list))
    u = _f64(np.stack(u_list))
    ns = f.shape[0]
    shape = f.shape[1:]
    dim, n, _ = _shape_args(shape)
    a = np.empty(shape)
    b = np.empty(shape)
    dl = ctypes.c_double(0.0)
    lib.orc_train_features(dim, n.ctypes.data_as(_ip), ns, _ptr(f), _ptr(u), _ptr(a), _ptr(b), ctypes.byref(dl))
    return a, b, dl.value


def train_loss(theta, M, alpha, beta, delta) -> float:
    lib = _load()
    alpha = _f64(alpha)
    beta = _f64(beta)
    dim, n, _ = _shape_args(alpha.shape)
    theta = _f64(theta)
    return lib.orc_train_loss(dim, n.ctypes.data_as(_ip), int(M), _ptr(theta), _ptr(alpha), _ptr(beta), float(delta))


def train_closed_form(M, alpha, beta) -> np.ndarray:
    lib = _load()
    alpha = _f64(alpha)
    beta = _f64(beta)
    check_modes(alpha.shape, M)
    dim, n, _ = _shape_args(alpha.shape)
    theta = np.zeros(num_weights(dim, M))
    lib.orc_train_closed_form(dim, n.ctypes.data_as(_ip), int(M), _ptr(alpha), _ptr(beta), _ptr(theta))
    return theta


# ---- linear elasticity, d = 3, c = 3 (Sec. 5.2); fields planar (3, *grid) ----

def lame(E, nu):
    """Lame coefficients of an isotropic material from Young's modulus and Poisson's ratio."""
    E = np.asarray(E, dtype=np.float64)
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def el_element_matrix(shape, lam, mu, L0=1.0, h=None):
    lib = _load()
    _, n, hh = _shape_args(shape, L0, h)
    K = np.zeros((24, 24))
    lib.orc_el_element_matrix(n.ctypes.data_as(_ip), _ptr(hh), float(lam), float(mu), _ptr(K))
    return K


def el_apply(lam, mu, u, L0=1.0, h=None):
    lib = _load()
    lam, mu, u = _f64(lam), _f64(mu), _f64(u)
    _, n, hh = _shape_args(lam.shape, L0, h)
    y = np.zeros_like(u)
    lib.orc_el_apply(n.ctypes.data_as(_ip), _ptr(hh), _ptr(lam), _ptr(mu), _ptr(u), _ptr(y))
    return y


def el_diag(lam, mu, L0=1.0, h=None):
    lib = _load()
    lam, mu = _f64(lam), _f64(mu)
    _, n, hh = _shape_args(lam.shape, L0, h)
    dg = np.zeros((3,) + lam.shape)
    lib.orc_el_diag(n.ctypes.data_as(_ip), _ptr(hh), _ptr(lam), _ptr(mu), _ptr(dg))
    return dg


def el_rhs(lam, mu, eps, L0=1.0, h=None):
    lib = _load()
    lam, mu = _f64(lam), _f64(mu)
    _, n, hh = _shape_args(lam.shape, L0, h)
    f = np.zeros((3,) + lam.shape)
    lib.orc_el_rhs(n.ctypes.data_as(_ip), _ptr(hh), _ptr(lam), _ptr(mu), _ptr(_f64(eps)), _ptr(f))
    return f


def el_stress_average(lam, mu, eps, u, L0=1.0, h=None):
    lib = _load()
    lam, mu = _f64(lam), _f64(mu)
    _, n, hh = _shape_args(lam.shape, L0, h)
    out = np.zeros(6)
    lib.orc_el_stress_average(n.ctypes.data_as(_ip), _ptr(hh), _ptr(lam), _ptr(mu), _ptr(_f64(eps)), _ptr(_f64(u)),
                              _ptr(out))
    return out


def el_pcg(lam, mu, f, kind="jacobi", rtol=1e-10, max_iter=100000, L0=1.0, h=None, table=None):
    """Algorithm 1 for the elastic operator (kind "none", "jacobi" or "uno"
    with a table of uno3_table); returns (u, passes)."""
    lib = _load()
    lam, mu, f = _f64(lam), _f64(mu), _f64(f)
    _, n, hh = _shape_args(lam.shape, L0, h)
    u = np.zeros_like(f)
    k = {"none": 0, "jacobi": 1, "uno": 2}[kind]
    tab = _f64(table) if k == 2 else np.zeros(1)
    if k == 2:
        assert tab.shape == (6,) + lam.shape
    it = lib.orc_el_pcg(n.ctypes.data_as(_ip), _ptr(hh), _ptr(lam), _ptr(mu), _ptr(f), _ptr(u), k, _ptr(tab),
                        float(rtol), int(max_iter))
    return u, int(it)


def el_effective_stiffness(lam, mu, solutions, loads=None, L0=1.0, h=None):
    """6 x 6 Mandel stiffness from the stress averages of the six unit Mandel
    strain loads (column j = <D (eps_j + eps(u_j))>)."""
    loads = np.eye(6) if loads is None else np.asarray(loads, dtype=np.float64)
    S = np.stack([el_stress_average(lam, mu, e, u, L0, h) for e, u in zip(loads, solutions)], axis=1)
    return S @ np.linalg.inv(loads.T)



# ---- UNO preconditioner and its training for c = 3 (App. B) ----

def psi3(w) -> np.ndarray:
    """(q1..q6) = unique entries of psi(w) = L L^T (eq. local-param-3)."""
    lib = _load()
    w = _f64(w)
    q = np.zeros(6)
    lib.orc_psi3(_ptr(w), _ptr(q))
    return q


def q_matrix(q) -> np.ndarray:
    """3 x 3 matrix of the table entries (q1, q2, q3, q4, q5, q6)."""
    q1, q2, q3, q4, q5, q6 = q
    return np.array([[q1, q3, q6], [q3, q2, q5], [q6, q5, q4]])


def num_weights3(M: int) -> int:
    return 6 * num_weights(3, M)


def uno3_table(shape, M, theta) -> np.ndarray:
    lib = _load()
    check_modes(shape, M)
    theta = _f64(theta)
    assert theta.size == num_weights3(M)
    _, n, _ = _shape_args(shape)
    t = np.zeros((6,) + tuple(shape))
    lib.orc_uno3_table(n.ctypes.data_as(_ip), int(M), _ptr(theta), _ptr(t))
    return t


def uno3_apply(table, r, return_imag=False):
    lib = _load()
    table, r = _f64(table), _f64(r)
    _, n, _ = _shape_args(r.shape[1:])
    s = np.zeros_like(r)
    im = lib.orc_uno3_apply(n.ctypes.data_as(_ip), _ptr(table), _ptr(r), _ptr(s))
    return (s, im) if return_imag else s


def train3_features(f_list, u_list):
    """(alpha (6, grid), beta (6, grid), delta) over the full Fourier grid."""
    lib = _load()
    f = _f64(np.stack(f_list))
    u = _f64(np.stack(u_list))
    ns = f.shape[0]
    shape = f.shape[2:]
    _, n, _ = _shape_args(shape)
    a = np.zeros((6,) + shape)
    b = np.zeros((6,) + shape)
    dl = ctypes.c_double(0.0)
    lib.orc_train3_features(n.ctypes.data_as(_ip), ns, _ptr(f), _ptr(u), _ptr(a), _ptr(b), ctypes.byref(dl))
    return a, b, dl.value


def train3_loss(theta, M, alpha, beta, delta) -> float:
    lib = _load()
    alpha, beta, theta = _f64(alpha), _f64(beta), _f64(theta)
    _, n, _ = _shape_args(alpha.shape[1:])
    return lib.orc_train3_loss(n.ctypes.data_as(_ip), int(M), _ptr(theta), _ptr(alpha), _ptr(beta), float(delta))


def train3_grad_hess(theta, M, alpha, beta, hess=True):
    lib = _load()
    alpha, beta, theta = _f64(alpha), _f64(beta), _f64(theta)
    _, n, _ = _shape_args(alpha.shape[1:])
    nw = num_weights3(M)
    g = np.zeros(nw)
    H = np.zeros((nw, nw)) if hess else None
    lib.orc_train3_grad_hess(n.ctypes.data_as(_ip), int(M), _ptr(theta), _ptr(alpha), _ptr(beta), _ptr(g),
                             _ptr(H) if hess else None)
    return (g, H) if hess else g


def train3_init(M, alpha, beta) -> np.ndarray:
    """Start of the Newton iteration: every slot isotropic, psi = a I, with a
    the best single scalar multiple of the identity for the data."""
    a_iso = (beta[0].sum() + beta[1].sum() + beta[3].sum()) / (2.0 * (alpha[0].sum() + alpha[1].sum() + alpha[3].sum()))
    w = np.sqrt(max(a_iso, 1e-300) / 2.0)
    theta = np.zeros(num_weights3(M))
    theta.reshape(-1, 6)[:, [0, 1, 3]] = w
    return theta


def train3_newton(M, alpha, beta, delta, theta0=None, epochs=100, gtol=1e-10):
    """Algorithm 4 (second-order training) with a Levenberg-Marquardt
    safeguard: the step solves (H + lam I) d = -g, lam shrinks after a step
    that lowers the loss and grows (the step is retried) otherwise.  With
    lam -> 0 it is the Newton-Raphson step of the paper.  Stops when the
    gradient has fallen by gtol or two steps no longer lower the loss beyond
    rounding.  Returns (theta, losses)."""
    theta = train3_init(M, alpha, beta) if theta0 is None else _f64(theta0).copy()
    L = train3_loss(theta, M, alpha, beta, delta)
    losses = [L]
    lam = None
    g0 = None
    for _ in range(epochs):
        g, H = train3_grad_hess(theta, M, alpha, beta)
        g0 = np.abs(g).max() if g0 is None else g0
        if np.abs(g).max() <= gtol * g0:
            break
        if len(losses) >= 3 and losses[-3] - losses[-1] <= 1e-14 * abs(losses[-1]):
            break  # stationary to rounding
        if lam is None:
            lam = 1e-6 * np.abs(np.diag(H)).max()
        while True:
            d = np.linalg.solve(H + lam * np.eye(H.shape[0]), -g)
            Ln = train3_loss(theta + d, M, alpha, beta, delta)
            if Ln <= L:
                theta, L = theta + d, Ln
                lam = max(lam / 3.0, 1e-300)
                break
            lam *= 4.0
            if lam > 1e300:
                return theta, losses
        losses.append(L)
    return theta, losses
