"""GPU: the allocation-free solve (pcg_solve_noalloc, workspace in the
library's fixed device array) gives bitwise the results of pcg_solve, call
after call on one device with the array keeping the previous call's
contents (each next problem smaller or of another kind), and refuses a
problem that does not fit."""
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


def _kappa(shape, seed, r=(2, 4)):
    ph, _ = si.rsa_inclusions(shape, r[0], r[1], 0.25, seed)
    return si.two_phase_kappa(ph, 1.0, 100.0)


def _case(uno, shape, kind, M, path, op, seed):
    kap = T(_kappa(shape, seed))
    p = None
    if kind == "uno":
        th = si.random_theta(uno.num_weights(len(shape), M), seed + 1, scale=0.05, spread=0.2)
        p = uno.UnoPrecond.create(shape, M, th)
        if path:
            p.set_path(path)
    g = np.zeros(len(shape))
    g[0] = 1.0
    return dict(kappa=kap, macro_load=g, kind=kind, precond=p, rtol=1e-8, max_iter=5000, op_dtype=op,
                prec_dtype=op, history=True)


# one after another: the headline grid, then smaller grids and other kinds
SEQUENCE = [
    ((64, 64, 64), "uno", 12, 0, torch.float64, 1),
    ((24, 20, 16), "jacobi", 0, 0, torch.float64, 2),
    ((32, 32, 32), "uno", 4, 0, torch.float32, 3),
    ((40, 36), "uno", 5, 1, torch.float64, 4),
    ((20, 12, 16), "none", 0, 0, torch.float64, 5),
]


def _compare(uno, kw, tag):
    ua, ia, ha = uno.pcg_solve(noalloc=True, **kw)
    ub, ib, hb = uno.pcg_solve(**kw)
    print("noalloc", tag, ia["iters"], ib["iters"], flush=True)
    assert ia["converged"] and ib["converged"]
    assert ia == ib, (tag, ia, ib)
    assert np.array_equal(ha, hb), tag
    assert torch.equal(ua, ub), "%s: the allocation-free solve differs from pcg_solve" % tag


def test_noalloc_equals_pcg_solve_call_after_call(uno):
    for case in SEQUENCE:
        _compare(uno, _case(uno, *case), case[:5])


def test_noalloc_repeat_smaller_after_larger(uno):
    """Two calls in a row, the second smaller, each against pcg_solve; the
    first call's contents remain in the array."""
    big = _case(uno, (48, 40, 32), "uno", 6, 0, torch.float64, 7)
    small = _case(uno, (16, 12, 10), "uno", 2, 0, torch.float64, 8)
    _compare(uno, big, "big")
    _compare(uno, small, "small")
    _compare(uno, big, "big again")


def test_noalloc_refuses_a_problem_that_does_not_fit(uno):
    kap = torch.ones((96, 96, 96), dtype=torch.float64, device=DEV)
    with pytest.raises(uno.UnoError) as e:
        uno.pcg_solve(kap, macro_load=[1.0, 0.0, 0.0], kind="jacobi", noalloc=True)
    assert e.value.status == -2  # UNO_ERR_SHAPE
