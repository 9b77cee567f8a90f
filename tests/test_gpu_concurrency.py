"""GPU: solves on different streams from different host threads give
bitwise the results of the same solves run one after another.

Every CG workspace (vectors, partials, loop states, the pinned host copy of
the states) belongs to one (device, grid, stream); a solve holds it from
start to end.  Cases: two grids at once, and one grid with two different
preconditioners at once (UNO and Jacobi, and two UNO tables)."""
import threading

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


def _kappa(shape, seed):
    ph, _ = si.rsa_inclusions(shape, 2, 4, 0.25, seed)
    return si.two_phase_kappa(ph, 1.0, 100.0)


def _precond(uno, shape, M, seed):
    th = si.random_theta(uno.num_weights(len(shape), M), seed, scale=0.05, spread=0.2)
    return uno.UnoPrecond.create(shape, M, th)


def _job(uno, shape, kind, M, seed, op=torch.float64):
    kap = T(_kappa(shape, seed))
    p = _precond(uno, shape, M, seed + 1) if kind == "uno" else None
    loads = np.eye(len(shape))

    def run():
        u, infos = uno.pcg_solve_batch(kap, macro_loads=loads, kind=kind, precond=p, rtol=1e-8, max_iter=20000,
                                       op_dtype=op, prec_dtype=op)
        return u, [i["iters"] for i in infos]
    return run


def _concurrent(jobs, rounds):
    """Each job on a stream of its own in a thread of its own, started
    together; results per round."""
    streams = [torch.cuda.Stream() for _ in jobs]
    torch.cuda.synchronize()
    out = [[None] * len(jobs) for _ in range(rounds)]
    errs = []

    for rd in range(rounds):
        bar = threading.Barrier(len(jobs))

        def work(i):
            try:
                with torch.cuda.stream(streams[i]):
                    bar.wait()
                    u, it = jobs[i]()
                    streams[i].synchronize()
                    out[rd][i] = (u.clone(), it)
                    streams[i].synchronize()
            except Exception as e:  # surfaced below
                errs.append(e)

        th = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
    assert not errs, errs
    return out


CASES = {
    "two_grids": [((24, 20, 16), "uno", 3, 11), ((40, 36), "uno", 5, 21), ((18, 16, 20), "jacobi", 0, 31)],
    "one_grid_uno_and_jacobi": [((24, 20, 16), "uno", 3, 41), ((24, 20, 16), "jacobi", 0, 41)],
    "one_grid_two_tables": [((24, 20, 16), "uno", 3, 51), ((24, 20, 16), "uno", 4, 52)],
    "fp32_and_fp64": [((24, 20, 16), "uno", 3, 61, torch.float32), ((24, 20, 16), "uno", 3, 61)],
}


@pytest.mark.parametrize("case", list(CASES))
def test_concurrent_streams_equal_sequential(uno, case):
    print("concurrency", case, flush=True)
    jobs = [_job(uno, *c) for c in CASES[case]]
    ref = []
    for j in jobs:  # one after another on the current stream
        u, it = j()
        torch.cuda.synchronize()
        ref.append((u.clone(), it))
    for rd, res in enumerate(_concurrent(jobs, rounds=3)):
        for i, (u, it) in enumerate(res):
            assert it == ref[i][1], (case, rd, i, it, ref[i][1])
            assert torch.equal(u, ref[i][0]), "%s round %d job %d differs from its sequential run" % (case, rd, i)
