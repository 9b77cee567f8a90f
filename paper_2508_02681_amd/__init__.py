"""Python binding of the gfx950 UNO-CG library (libunocg.so, C ABI in
include/unocg.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  Tensors must be contiguous CUDA (HIP) tensors; work is
enqueued on torch's current stream.  The binding refuses to run when the
library has not been built (``python -m paper_2508_02681_amd.build``).

Entry points mirror the C ABI: fe_apply, jac_precond_apply, uno_macro_rhs,
UnoPrecond (uno_precond_create / _create_fans / _apply / _destroy),
pcg_solve, effective_tensor, uno_train_accumulate, uno_train_fit.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libunocg.so")

UNO_F64, UNO_F32, UNO_BF16 = 0, 1, 2
UNO_PREC_NONE, UNO_PREC_JACOBI, UNO_PREC_UNO = 0, 1, 2
KT_NONE, KT_MATVEC, KT_UPDATE, KT_FFT_FWD, KT_FFT_MID, KT_FFT_INV, KT_APPLY = 0, 1, 2, 3, 4, 5, 6
STATUS = {0: "UNO_OK", -1: "UNO_ERR_ARG", -2: "UNO_ERR_SHAPE", -3: "UNO_ERR_NOT_SPD",
          -4: "UNO_ERR_BREAKDOWN", -5: "UNO_ERR_DEVICE", -6: "UNO_ERR_NOMEM"}


class UnoError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(status, "?"), status))


class uno_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("L0", ctypes.c_double)]


class uno_material(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_void_p), ("dtype", ctypes.c_int)]


class uno_solve_opts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("uno", ctypes.c_void_p), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("op_t", ctypes.c_int), ("prec_t", ctypes.c_int),
                ("graph_chunk", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


class uno_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("r0_norm", ctypes.c_double)]


_lib = None


def lib():
    """Loads libunocg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libunocg.so is not built (run python -m paper_2508_02681_amd.build); "
                           "there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, f64, i = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    G, Mt = P(uno_grid), P(uno_material)
    sig = {
        "uno_status_string": ([i], ctypes.c_char_p),
        "fe_apply": ([G, Mt, vp, vp, i, vp], i),
        "jac_precond_apply": ([G, Mt, vp, vp, i, vp], i),
        "uno_macro_rhs": ([G, Mt, P(f64), vp, i, vp], i),
        "uno_precond_create": ([G, i32, P(f64), i64, f64, i, P(vp)], i),
        "el_uno_precond_create": ([G, i32, P(f64), i64, f64, P(vp)], i),
        "pcg_solve_many": ([i32, P(uno_problem), P(uno_solve_opts), vp], i),
        "el_uno_train_accumulate": ([G, i32, vp, vp, f64, vp, vp, vp], i),
        "el_uno_train_fit": ([G, i32, vp, vp, i32, P(f64), i64, P(f64), vp], i),
        "uno_precond_create_fans": ([G, f64, i, P(vp)], i),
        "uno_precond_apply": ([vp, vp, vp, i, vp], i),
        "uno_precond_table": ([vp, P(f64), i64], i),
        "uno_precond_set_path": ([vp, i32], i),
        "uno_precond_destroy": ([vp], i),
        "pcg_solve": ([G, Mt, P(f64), vp, vp, P(uno_solve_opts), P(uno_solve_info), P(f64), vp], i),
        "pcg_solve_noalloc": ([G, Mt, P(f64), vp, vp, P(uno_solve_opts), P(uno_solve_info), P(f64), vp], i),
        "pcg_solve_batch": ([G, Mt, i32, i32, P(f64), vp, vp, P(uno_solve_opts), P(uno_solve_info), vp], i),
        "effective_tensor": ([G, Mt, i32, P(f64), vp, P(f64), vp], i),
        "effective_tensor_batch": ([G, Mt, i32, i32, P(f64), vp, P(f64), vp], i),
        "effective_tensor_grad": ([G, i32, P(f64), vp, P(f64), vp, vp], i),
        "el_apply": ([G, vp, vp, vp, vp, vp], i),
        "el_macro_rhs": ([G, vp, vp, P(f64), vp, vp], i),
        "el_pcg_solve": ([G, vp, vp, i32, i32, P(f64), vp, P(uno_solve_opts), P(uno_solve_info), vp], i),
        "el_effective_stiffness": ([G, vp, vp, i32, P(f64), vp, P(f64), vp], i),
        "uno_train_accumulate": ([G, i32, vp, vp, f64, vp, vp, vp], i),
        "uno_train_fit": ([G, i32, vp, vp, P(f64), i64, vp], i),
        "uno_train_loss_grad": ([G, i32, vp, vp, P(f64), i64, P(f64), P(f64), vp], i),
        "uno_timing_enable": ([i32], i),
        "uno_timing_read": ([P(f64), P(i64)], i),
        "uno_shutdown": ([], i),
        "uno_autotune_operator": ([G, i32, i32, i, vp, P(i32), P(i32), P(i32), P(f64)], i),
        "uno_set_operator_shape": ([G, i32, i32, i, i32, i32, i32], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(st, where):
    if st != 0:
        raise UnoError(st, where)


def _dt(t: torch.dtype) -> int:
    if t == torch.float64:
        return UNO_F64
    if t == torch.float32:
        return UNO_F32
    if t == torch.bfloat16:
        return UNO_BF16
    raise TypeError("unsupported dtype %s" % t)


def make_grid(shape, L0=1.0) -> uno_grid:
    shape = tuple(int(s) for s in shape)
    if len(shape) not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    g = uno_grid()
    g.dim = len(shape)
    for b in range(3):
        g.n[b] = shape[b] if b < len(shape) else 1
    g.L0 = float(L0)
    return g


def _dev(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mat(kappa: torch.Tensor) -> uno_material:
    m = uno_material()
    m.kappa = _dev(kappa, "kappa")
    m.dtype = _dt(kappa.dtype)
    return m


def fe_apply(kappa: torch.Tensor, u: torch.Tensor, y: torch.Tensor | None = None, L0=1.0) -> torch.Tensor:
    """y = A(kappa) u (matrix-free periodic FE operator)."""
    if y is None:
        y = torch.empty_like(u)
    g = make_grid(kappa.shape, L0)
    _check(lib().fe_apply(ctypes.byref(g), ctypes.byref(_mat(kappa)), _dev(u, "u", kappa.dtype),
                          _dev(y, "y", kappa.dtype), _dt(u.dtype), _stream()), "fe_apply")
    return y


def jac_precond_apply(kappa: torch.Tensor, r: torch.Tensor, s: torch.Tensor | None = None, L0=1.0):
    if s is None:
        s = torch.empty_like(r)
    g = make_grid(kappa.shape, L0)
    _check(lib().jac_precond_apply(ctypes.byref(g), ctypes.byref(_mat(kappa)), _dev(r, "r", kappa.dtype),
                                   _dev(s, "s", kappa.dtype), _dt(r.dtype), _stream()), "jac_precond_apply")
    return s


def uno_macro_rhs(kappa: torch.Tensor, gbar, out: torch.Tensor | None = None, dtype=torch.float64, L0=1.0):
    if out is None:
        out = torch.empty(kappa.shape, dtype=dtype, device=kappa.device)
    g = make_grid(kappa.shape, L0)
    gb = np.ascontiguousarray(gbar, dtype=np.float64)
    if gb.size != len(kappa.shape):
        raise ValueError("gbar needs one value per axis")
    _check(lib().uno_macro_rhs(ctypes.byref(g), ctypes.byref(_mat(kappa)),
                               gb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _dev(out, "f"),
                               _dt(out.dtype), _stream()), "uno_macro_rhs")
    return out


def num_weights(dim: int, M: int) -> int:
    return (2 * M + 1) ** (dim - 1) * (M + 1)


class UnoPrecond:
    """Owns a uno_precond handle (device table + scratch)."""

    def __init__(self, handle, shape, L0):
        self._h = handle
        self.shape = tuple(shape)
        self.L0 = L0

    @classmethod
    def create(cls, shape, M, theta, eps_spd=1e-300, table_dtype=torch.float64, L0=1.0):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        g = make_grid(shape, L0)
        h = ctypes.c_void_p()
        _check(lib().uno_precond_create(ctypes.byref(g), int(M), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        th.size, float(eps_spd), _dt(table_dtype), ctypes.byref(h)),
               "uno_precond_create")
        return cls(h, shape, L0)

    @classmethod
    def create_elastic(cls, shape, M, theta, eps_spd=1e-300, L0=1.0):
        """Three nodal DOF (elasticity): theta holds 6 weights per slot
        (psi(w) = L L^T, L = [w1 0 0; w3 w2 0; w6 w5 w4]); apply() takes
        3 x grid vectors."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        g = make_grid(shape, L0)
        h = ctypes.c_void_p()
        _check(lib().el_uno_precond_create(ctypes.byref(g), int(M), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           th.size, float(eps_spd), ctypes.byref(h)), "el_uno_precond_create")
        return cls(h, shape, L0)

    @classmethod
    def fans(cls, shape, kappa_ref, table_dtype=torch.float64, L0=1.0):
        g = make_grid(shape, L0)
        h = ctypes.c_void_p()
        _check(lib().uno_precond_create_fans(ctypes.byref(g), float(kappa_ref), _dt(table_dtype), ctypes.byref(h)),
               "uno_precond_create_fans")
        return cls(h, shape, L0)

    @property
    def handle(self):
        return self._h

    def apply(self, r: torch.Tensor, s: torch.Tensor | None = None) -> torch.Tensor:
        if s is None:
            s = torch.empty_like(r)
        _check(lib().uno_precond_apply(self._h, _dev(r, "r"), _dev(s, "s", r.dtype), _dt(r.dtype), _stream()),
               "uno_precond_apply")
        return s

    PATH_AUTO, PATH_SPECTRAL, PATH_LEARNED, PATH_FUSED = 0, 1, 2, 3

    def set_path(self, path: int):
        """0 auto, 1 full spectral passes, 2 learned-mode passes (FP64)."""
        _check(lib().uno_precond_set_path(self._h, int(path)), "uno_precond_set_path")

    def table(self) -> np.ndarray:
        shp = list(self.shape)
        shp[-1] = shp[-1] // 2 + 1
        out = np.empty(shp, dtype=np.float64)
        _check(lib().uno_precond_table(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               "uno_precond_table")
        return out

    def close(self):
        if self._h is not None and self._h.value:
            lib().uno_precond_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve(kappa: torch.Tensor, macro_load=None, rhs: torch.Tensor | None = None, u: torch.Tensor | None = None,
              kind="jacobi", precond: UnoPrecond | None = None, rtol=1e-6, max_iter=100000,
              op_dtype=torch.float64, prec_dtype=torch.float64, graph_chunk=0, history=False, L0=1.0,
              noalloc=False, use_graphs=False):
    """Preconditioned CG (Algorithm 1/2).  Returns (u, info dict[, hist]).
    noalloc: the allocation-free entry point (workspace in the library's
    fixed device array; raises UnoError SHAPE when the problem does not fit)."""
    kinds = {"none": UNO_PREC_NONE, "jacobi": UNO_PREC_JACOBI, "uno": UNO_PREC_UNO}
    g = make_grid(kappa.shape, L0)
    if u is None:
        u = torch.zeros(kappa.shape, dtype=torch.float64, device=kappa.device)
    o = uno_solve_opts()
    o.kind = kinds[kind]
    o.uno = precond.handle if (precond is not None and kind == "uno") else None
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.op_t = _dt(op_dtype)
    o.prec_t = _dt(prec_dtype)
    o.graph_chunk = int(graph_chunk)
    o.use_graphs = 1 if use_graphs else 0
    info = uno_solve_info()
    ml = None
    if macro_load is not None:
        ml = np.ascontiguousarray(macro_load, dtype=np.float64)
        if ml.size != len(kappa.shape):
            raise ValueError("macro_load needs one value per axis")
    hist = np.zeros(max_iter + 1) if history else None
    entry = lib().pcg_solve_noalloc if noalloc else lib().pcg_solve
    st = entry(
        ctypes.byref(g), ctypes.byref(_mat(kappa)),
        ml.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ml is not None else None,
        _dev(rhs, "rhs", torch.float64) if rhs is not None else None,
        _dev(u, "u", torch.float64), ctypes.byref(o), ctypes.byref(info),
        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if hist is not None else None, _stream())
    _check(st, "pcg_solve_noalloc" if noalloc else "pcg_solve")
    d = dict(iters=info.iters, converged=bool(info.converged), rel_res=info.rel_res,
             true_rel_res=info.true_rel_res, r0_norm=info.r0_norm)
    if history:
        return u, d, hist[: info.iters + 1].copy()
    return u, d


def _opts(kind, precond, rtol, max_iter, op_dtype, prec_dtype, graph_chunk, use_graphs=False):
    kinds = {"none": UNO_PREC_NONE, "jacobi": UNO_PREC_JACOBI, "uno": UNO_PREC_UNO}
    o = uno_solve_opts()
    o.kind = kinds[kind]
    o.uno = precond.handle if (precond is not None and kind == "uno") else None
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.op_t = _dt(op_dtype)
    o.prec_t = _dt(prec_dtype)
    o.graph_chunk = int(graph_chunk)
    o.use_graphs = 1 if use_graphs else 0
    return o


def pcg_solve_batch(kappa: torch.Tensor, macro_loads=None, rhs: torch.Tensor | None = None,
                    u: torch.Tensor | None = None, kind="jacobi", precond: UnoPrecond | None = None, rtol=1e-6,
                    max_iter=100000, op_dtype=torch.float64, prec_dtype=torch.float64, graph_chunk=0,
                    kappa_per_rhs=False, L0=1.0, use_graphs=False):
    """nrhs solves carried together by every pass kernel: the load cases of
    one conductivity field (kappa: grid), or with kappa_per_rhs one field per
    right-hand side (kappa: nrhs x grid).  macro_loads: nrhs x d (host) or
    rhs: nrhs x grid (device).  Returns (u (nrhs x grid), [info])."""
    shape = tuple(kappa.shape[1:]) if kappa_per_rhs else tuple(kappa.shape)
    g = make_grid(shape, L0)
    d = len(shape)
    ml = None
    if macro_loads is not None:
        ml = np.ascontiguousarray(macro_loads, dtype=np.float64).reshape(-1, d)
        nrhs = ml.shape[0]
    else:
        nrhs = rhs.shape[0]
    if kappa_per_rhs and kappa.shape[0] != nrhs:
        raise ValueError("kappa_per_rhs needs one field per right-hand side")
    if u is None:
        u = torch.zeros((nrhs,) + shape, dtype=torch.float64, device=kappa.device)
    if tuple(u.shape) != (nrhs,) + shape:
        raise ValueError("u must be nrhs x grid")
    o = _opts(kind, precond, rtol, max_iter, op_dtype, prec_dtype, graph_chunk, use_graphs)
    infos = (uno_solve_info * nrhs)()
    st = lib().pcg_solve_batch(
        ctypes.byref(g), ctypes.byref(_mat(kappa)), 1 if kappa_per_rhs else 0, nrhs,
        ml.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ml is not None else None,
        _dev(rhs, "rhs", torch.float64) if rhs is not None else None,
        _dev(u, "u", torch.float64), ctypes.byref(o), infos, _stream())
    _check(st, "pcg_solve_batch")
    return u, [dict(iters=I.iters, converged=bool(I.converged), rel_res=I.rel_res, true_rel_res=I.true_rel_res,
                    r0_norm=I.r0_norm) for I in infos]


def effective_tensor(kappa: torch.Tensor, loads, solutions: torch.Tensor, L0=1.0) -> np.ndarray:
    """kappa_bar (d x d) from the solutions of the d load cases."""
    g = make_grid(kappa.shape, L0)
    ld = np.ascontiguousarray(loads, dtype=np.float64)
    d = len(kappa.shape)
    out = np.zeros((d, d))
    _check(lib().effective_tensor(ctypes.byref(g), ctypes.byref(_mat(kappa)), ld.shape[0],
                                  ld.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _dev(solutions, "solutions", torch.float64),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()), "effective_tensor")
    return out


def effective_tensor_batch(kappas: torch.Tensor, loads, solutions: torch.Tensor, L0=1.0) -> np.ndarray:
    """kappa_bar (nmat x d x d) of nmat microstructures (kappas: nmat x grid)
    from their solutions (nmat * d x grid, the d load cases of field m at
    m d .. m d + d - 1), one read-back for all."""
    nm = kappas.shape[0]
    shape = tuple(kappas.shape[1:])
    g = make_grid(shape, L0)
    ld = np.ascontiguousarray(loads, dtype=np.float64)
    d = len(shape)
    if tuple(solutions.shape) != (nm * ld.shape[0],) + shape:
        raise UnoError(-1, "effective_tensor_batch (solutions must be (nmat * nload,) + grid)")
    out = np.zeros((nm, d, d))
    _check(lib().effective_tensor_batch(ctypes.byref(g), ctypes.byref(_mat(kappas)), nm, ld.shape[0],
                                        ld.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        _dev(solutions, "solutions", torch.float64),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
           "effective_tensor_batch")
    return out


def effective_tensor_grad(shape, loads, solutions: torch.Tensor, weights=None, out: torch.Tensor | None = None,
                          L0=1.0) -> torch.Tensor:
    """d kappa_bar_ij / d kappa_e for every voxel (d x d x grid, device), or
    with weights (d x d) the vector-Jacobian product sum_ij w_ij d kappa_bar_ij
    / d kappa_e (grid).  solutions: the load cases' solutions (d x grid)."""
    shape = tuple(shape)
    g = make_grid(shape, L0)
    d = len(shape)
    ld = np.ascontiguousarray(loads, dtype=np.float64)
    if ld.shape != (d, d):
        raise ValueError("need d loads of d components")
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64).reshape(d, d)
    if out is None:
        oshape = shape if w is not None else (d, d) + shape
        out = torch.empty(oshape, dtype=torch.float64, device=solutions.device)
    _check(lib().effective_tensor_grad(ctypes.byref(g), d, ld.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       _dev(solutions, "solutions", torch.float64),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if w is not None else None,
                                       _dev(out, "out", torch.float64), _stream()), "effective_tensor_grad")
    return out


class EffectiveConductivity(torch.autograd.Function):
    """kappa_bar(kappa) with a hand-written backward: forward solves the d
    unit load cases together (UNO-CG or Jacobi-CG), backward contracts the
    incoming gradient with the element energy densities of the saved
    solutions (the cell problem is self-adjoint: no adjoint solve, no stored
    CG iterates)."""

    @staticmethod
    def forward(ctx, kappa, kind="jacobi", precond=None, rtol=1e-10):
        d = kappa.dim()
        loads = np.eye(d)
        u, infos = pcg_solve_batch(kappa.detach(), macro_loads=loads, kind=kind, precond=precond, rtol=rtol)
        if not all(i["converged"] for i in infos):
            raise UnoError("effective conductivity: a cell problem did not converge")
        kb = effective_tensor(kappa.detach(), loads, u)
        ctx.save_for_backward(u)
        ctx.shape = tuple(kappa.shape)
        return torch.tensor(kb, dtype=torch.float64, device=kappa.device)

    @staticmethod
    def backward(ctx, grad_out):
        (u,) = ctx.saved_tensors
        d = len(ctx.shape)
        w = grad_out.detach().double().cpu().numpy()
        gk = effective_tensor_grad(ctx.shape, np.eye(d), u, weights=w)
        return gk, None, None, None


def uno_train_loss_grad(shape, M, alpha: torch.Tensor, beta: torch.Tensor, theta, L0=1.0):
    """(loss, dloss/dtheta) of the batch features alpha, beta (half spectrum,
    device) at theta; loss omits the constant (1/Ns) sum ||u_j||^2."""
    g = make_grid(tuple(shape), L0)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    grad = np.zeros_like(th)
    loss = ctypes.c_double(0.0)
    _check(lib().uno_train_loss_grad(ctypes.byref(g), int(M), _dev(alpha, "alpha", torch.float64),
                                     _dev(beta, "beta", torch.float64), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     th.size, ctypes.byref(loss), grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     _stream()), "uno_train_loss_grad")
    return loss.value, grad


class UnoTrainLoss(torch.autograd.Function):
    """Batch loss of the UNO weights (Algorithm 3) as a function of theta,
    with the hand-written backward of uno_train_loss_grad."""

    @staticmethod
    def forward(ctx, theta, shape, M, alpha, beta):
        loss, grad = uno_train_loss_grad(shape, M, alpha, beta, theta.detach().cpu().numpy())
        ctx.save_for_backward(torch.tensor(grad, dtype=theta.dtype, device=theta.device))
        return torch.tensor(loss, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None


# ---- linear elasticity, d = 3, c = 3: displacements (3, *grid) per load ----

def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def el_apply(lam: torch.Tensor, mu: torch.Tensor, u: torch.Tensor, y: torch.Tensor | None = None, L0=1.0):
    """y = A(lambda, mu) u (u, y: 3 x grid)."""
    g = make_grid(tuple(lam.shape), L0)
    if y is None:
        y = torch.empty_like(u)
    _check(lib().el_apply(ctypes.byref(g), _dev(lam, "lambda", torch.float64), _dev(mu, "mu", torch.float64),
                          _dev(u, "u", torch.float64), _dev(y, "y", torch.float64), _stream()), "el_apply")
    return y


def el_macro_rhs(lam: torch.Tensor, mu: torch.Tensor, strain, L0=1.0):
    g = make_grid(tuple(lam.shape), L0)
    f = torch.empty((3,) + tuple(lam.shape), dtype=torch.float64, device=lam.device)
    e = np.ascontiguousarray(strain, dtype=np.float64).reshape(6)
    _check(lib().el_macro_rhs(ctypes.byref(g), _dev(lam, "lambda", torch.float64), _dev(mu, "mu", torch.float64),
                              _dptr(e), _dev(f, "f", torch.float64), _stream()), "el_macro_rhs")
    return f


def el_pcg_solve(lam: torch.Tensor, mu: torch.Tensor, strains, u: torch.Tensor | None = None, kind="jacobi",
                 rtol=1e-6, max_iter=100000, graph_chunk=0, lame_per_rhs=False, L0=1.0,
                 precond: UnoPrecond | None = None, op_dtype=torch.float64, use_graphs=False):
    """CG, Jacobi-CG or UNO-CG (kind "uno" with a UnoPrecond.create_elastic)
    for nrhs macroscopic Mandel strains (nrhs x 6).
    lam, mu: grid (shared) or nrhs x grid (lame_per_rhs).  op_dtype
    torch.float32: the FP32 mode (UNO-CG).  Returns (u (nrhs x 3 x grid),
    [info])."""
    shape = tuple(lam.shape[1:]) if lame_per_rhs else tuple(lam.shape)
    g = make_grid(shape, L0)
    e = np.ascontiguousarray(strains, dtype=np.float64).reshape(-1, 6)
    nrhs = e.shape[0]
    if u is None:
        u = torch.zeros((nrhs, 3) + shape, dtype=torch.float64, device=lam.device)
    o = _opts(kind, precond, rtol, max_iter, op_dtype, op_dtype, graph_chunk, use_graphs)
    infos = (uno_solve_info * nrhs)()
    _check(lib().el_pcg_solve(ctypes.byref(g), _dev(lam, "lambda", torch.float64), _dev(mu, "mu", torch.float64),
                              1 if lame_per_rhs else 0, nrhs, _dptr(e), _dev(u, "u", torch.float64), ctypes.byref(o),
                              infos, _stream()), "el_pcg_solve")
    return u, [dict(iters=I.iters, converged=bool(I.converged), rel_res=I.rel_res, true_rel_res=I.true_rel_res,
                    r0_norm=I.r0_norm) for I in infos]


def el_effective_stiffness(lam: torch.Tensor, mu: torch.Tensor, strains, u: torch.Tensor, L0=1.0) -> np.ndarray:
    """6 x 6 Mandel effective stiffness from the six loads' solutions u (6 x 3 x grid)."""
    g = make_grid(tuple(lam.shape), L0)
    e = np.ascontiguousarray(strains, dtype=np.float64).reshape(6, 6)
    out = np.zeros((6, 6))
    _check(lib().el_effective_stiffness(ctypes.byref(g), _dev(lam, "lambda", torch.float64),
                                        _dev(mu, "mu", torch.float64), 6, _dptr(e), _dev(u, "u", torch.float64),
                                        _dptr(out), _stream()), "el_effective_stiffness")
    return out


class uno_problem(ctypes.Structure):
    _fields_ = [("grid", uno_grid), ("kappa", ctypes.c_void_p), ("nload", ctypes.c_int32),
                ("loads", ctypes.POINTER(ctypes.c_double)), ("u", ctypes.c_void_p), ("uno", ctypes.c_void_p),
                ("info", ctypes.POINTER(uno_solve_info))]


def pcg_solve_many(problems, kind="uno", rtol=1e-6, max_iter=100000, graph_chunk=0, L0=1.0,
                   op_dtype=torch.float64, prec_dtype=torch.float64, use_graphs=False):
    """Solves many problems of uneven sizes in one call.  problems: list of
    dicts with "kappa" (device grid tensor), "loads" (nload x dim), optional
    "u" (nload x grid, zero-initialized if absent) and "precond" (UnoPrecond
    of that grid, for kind "uno").  Returns ([u], [[info]])."""
    n = len(problems)
    arr = (uno_problem * n)()
    keep = []
    us, infos = [], []
    for i, P in enumerate(problems):
        kap = P["kappa"]
        shape = tuple(kap.shape)
        loads = np.ascontiguousarray(P["loads"], dtype=np.float64).reshape(-1, len(shape))
        nl = loads.shape[0]
        u = P.get("u")
        if u is None:
            u = torch.zeros((nl,) + shape, dtype=torch.float64, device=kap.device)
        inf = (uno_solve_info * nl)()
        pr = P.get("precond")
        arr[i].grid = make_grid(shape, L0)
        arr[i].kappa = _dev(kap, "kappa", torch.float64)
        arr[i].nload = nl
        arr[i].loads = loads.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        arr[i].u = _dev(u, "u", torch.float64)
        arr[i].uno = pr.handle if (pr is not None and kind == "uno") else None
        arr[i].info = inf
        keep += [loads, inf]
        us.append(u)
        infos.append(inf)
    o = _opts(kind, None, rtol, max_iter, op_dtype, prec_dtype, graph_chunk, use_graphs)
    st = lib().pcg_solve_many(n, arr, ctypes.byref(o), _stream())
    out = [[dict(iters=I.iters, converged=bool(I.converged), rel_res=I.rel_res, true_rel_res=I.true_rel_res)
            for I in inf] for inf in infos]
    if st != 0:
        err = UnoError(st, "pcg_solve_many")
        err.infos = out  # per-load records (which load cases broke down)
        raise err
    return us, out


def half_shape(shape):
    s = list(shape)
    s[-1] = s[-1] // 2 + 1
    return tuple(s)


def uno_train_accumulate(f: torch.Tensor, u: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, ns_total,
                         L0=1.0):
    """alpha, beta (half spectrum, float64) += features of the samples f, u (ns x shape)."""
    shape = tuple(f.shape[1:])
    g = make_grid(shape, L0)
    _check(lib().uno_train_accumulate(ctypes.byref(g), f.shape[0], _dev(f, "f", torch.float64),
                                      _dev(u, "u", torch.float64), float(ns_total), _dev(alpha, "alpha", torch.float64),
                                      _dev(beta, "beta", torch.float64), _stream()), "uno_train_accumulate")


def uno_train_fit(shape, M, alpha: torch.Tensor, beta: torch.Tensor, L0=1.0) -> np.ndarray:
    g = make_grid(shape, L0)
    th = np.zeros(num_weights(len(shape), M))
    _check(lib().uno_train_fit(ctypes.byref(g), int(M), _dev(alpha, "alpha", torch.float64),
                               _dev(beta, "beta", torch.float64), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               th.size, _stream()), "uno_train_fit")
    return th


def autotune_operator(shape, nrhs, kappa_per_rhs=False, dtype=torch.float64, L0=1.0) -> dict:
    """Measures the operator march's shapes for nrhs right-hand sides of
    this grid and records the fastest (used by later solves).  Returns
    dict(tz, ry, xb, us)."""
    g = make_grid(shape, L0)
    tz, ry, xb, us = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().uno_autotune_operator(ctypes.byref(g), int(nrhs), 1 if kappa_per_rhs else 0, _dt(dtype), _stream(),
                                       ctypes.byref(tz), ctypes.byref(ry), ctypes.byref(xb), ctypes.byref(us)),
           "uno_autotune_operator")
    return dict(tz=tz.value, ry=ry.value, xb=xb.value, us=us.value)


def set_operator_shape(shape, nrhs, tz, ry, xb, kappa_per_rhs=False, dtype=torch.float64, L0=1.0):
    """Records the operator march shape (tz, ry, xb) for nrhs right-hand
    sides of this grid, as autotune_operator would."""
    g = make_grid(shape, L0)
    _check(lib().uno_set_operator_shape(ctypes.byref(g), int(nrhs), 1 if kappa_per_rhs else 0, _dt(dtype), int(tz),
                                        int(ry), int(xb)), "uno_set_operator_shape")


def timing_enable(which: int):
    _check(lib().uno_timing_enable(int(which)), "uno_timing_enable")


def timing_read():
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().uno_timing_read(ctypes.byref(ms), ctypes.byref(n)), "uno_timing_read")
    return ms.value, n.value


def shutdown():
    _check(lib().uno_shutdown(), "uno_shutdown")


def el_uno_train_accumulate(f: torch.Tensor, u: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, ns_total,
                            L0=1.0):
    """Adds the c = 3 features of the pairs f, u (ns x 3 x grid) into alpha,
    beta (6 x n0 x n1 x (n2/2+1), device, zeroed by the caller)."""
    shape = tuple(f.shape[2:])
    g = make_grid(shape, L0)
    _check(lib().el_uno_train_accumulate(ctypes.byref(g), int(f.shape[0]), _dev(f, "f", torch.float64),
                                         _dev(u, "u", torch.float64), float(ns_total),
                                         _dev(alpha, "alpha", torch.float64), _dev(beta, "beta", torch.float64),
                                         _stream()), "el_uno_train_accumulate")


def el_uno_train_fit(shape, M, alpha: torch.Tensor, beta: torch.Tensor, max_epochs=200, L0=1.0):
    """Newton training (Algorithm 4) of the c = 3 weights; returns (theta, loss
    less its constant)."""
    g = make_grid(shape, L0)
    nw = 6 * num_weights(3, M)
    th = np.zeros(nw)
    loss = ctypes.c_double(0.0)
    _check(lib().el_uno_train_fit(ctypes.byref(g), int(M), _dev(alpha, "alpha", torch.float64),
                                  _dev(beta, "beta", torch.float64), int(max_epochs),
                                  th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nw, ctypes.byref(loss),
                                  _stream()), "el_uno_train_fit")
    return th, loss.value
