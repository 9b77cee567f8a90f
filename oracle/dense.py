"""Dense references on tiny grids (test infrastructure only).

* ``assemble(kappa)``: the stiffness matrix A as a dense array, column j being
  the oracle's element-loop apply to the unit vector e_j (Sec. 3.1: the
  entries are a(phi_j, phi_i)).
* ``bordered_solve(A, f)``: the discrete periodic solution with zero mean,
  from the bordered system [A 1; 1^T 0][u; lam] = [f; 0] solved by LAPACK.
  This is the plain definition of the discrete solution, independent of any
  iteration.
* ``operator_matrix(apply, n)``: dense matrix of any linear map (used for
  the preconditioner spectra of Sec. 4.2.3).
"""
from __future__ import annotations

import numpy as np

from . import fe_apply


def operator_matrix(apply, shape) -> np.ndarray:
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(np.asarray(apply(e.reshape(shape))).reshape(n))
    return np.stack(cols, axis=1)


def assemble(kappa, L0=1.0, h=None) -> np.ndarray:
    kappa = np.asarray(kappa, dtype=np.float64)
    return operator_matrix(lambda v: fe_apply(kappa, v, L0, h), kappa.shape)


def bordered_solve(A, f) -> np.ndarray:
    n = A.shape[0]
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = A
    B[:n, n] = 1.0
    B[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[:n] = np.asarray(f).reshape(n)
    sol = np.linalg.solve(B, rhs)
    return sol[:n]
