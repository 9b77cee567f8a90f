"""GPU: CG passes replayed from captured hipGraphs (use_graphs) give bitwise
the results of the same passes launched one by one: thermal UNO-CG (the
learned-mode flow and its fused variant, one load and batched), Jacobi-CG,
plain CG, 2D cells, elastic UNO-CG and Jacobi-CG, and the many-problem list.
Every solve replays its chunk graph many times, with the program's own eager
work and host synchronizations between the solves; each graph-mode solve is
checked against the eager one, on the default stream and on a stream of its
own, and again after the operands move (new tensors: the graphs are
recaptured) and after the preconditioner is replaced."""
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


def _precond(uno, shape, M, seed, path=0):
    th = si.random_theta(uno.num_weights(len(shape), M), seed, scale=0.05, spread=0.2)
    p = uno.UnoPrecond.create(shape, M, th)
    if path:
        p.set_path(path)
    return p


def _same(a, b, tag):
    ua, ia = a
    ub, ib = b
    assert [i["iters"] for i in ia] == [i["iters"] for i in ib], tag
    assert [i["rel_res"] for i in ia] == [i["rel_res"] for i in ib], tag
    assert torch.equal(ua, ub), "%s: graph-mode solution differs from the eager one" % tag


CASES = [
    ("uno learned, 3 loads", (24, 20, 16), "uno", 3, 2, 3),
    ("uno fused, 3 loads", (24, 20, 16), "uno", 3, 3, 3),
    ("uno learned, 1 load", (32, 32, 32), "uno", 4, 0, 1),
    ("jacobi, 3 loads", (24, 20, 16), "jacobi", 0, 0, 3),
    ("none, 1 load", (16, 12, 10), "none", 0, 0, 1),
    ("uno 2D, 2 loads", (40, 36), "uno", 5, 0, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_mode_equals_eager(uno, case):
    tag, shape, kind, M, path, nl = case
    print("graphs", tag, flush=True)
    kap = T(_kappa(shape, 71))
    p = _precond(uno, shape, M, 72, path) if kind == "uno" else None
    loads = np.eye(len(shape))[:nl]
    kw = dict(kind=kind, precond=p, rtol=1e-9, max_iter=20000)

    def run(graphs):
        u, infos = uno.pcg_solve_batch(kap, macro_loads=loads, use_graphs=graphs, **kw)
        return u.clone(), infos

    ref = run(False)
    for rep in range(3):  # replays of the cached graph, eager work between them
        _same(ref, run(True), "%s rep %d" % (tag, rep))
        torch.cuda.synchronize()
        _same(ref, run(False), "%s eager rep %d" % (tag, rep))
    # a stream of its own
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = run(True)
        s.synchronize()
    _same(ref, got, tag + " own stream")
    # moved operands: the graphs are recaptured
    kap2 = kap.clone()
    u2, i2 = uno.pcg_solve_batch(kap2, macro_loads=loads, use_graphs=True, **kw)
    _same(ref, (u2, i2), tag + " moved kappa")


def test_graph_mode_new_preconditioner(uno):
    """A preconditioner replaced by another (possibly at the same address)
    is not served from a graph recorded for the first."""
    shape = (24, 20, 16)
    kap = T(_kappa(shape, 73))
    loads = np.eye(3)
    for seed in (74, 75, 76):
        p = _precond(uno, shape, 3, seed)
        ref = uno.pcg_solve_batch(kap, macro_loads=loads, kind="uno", precond=p, rtol=1e-9)
        got = uno.pcg_solve_batch(kap, macro_loads=loads, kind="uno", precond=p, rtol=1e-9, use_graphs=True)
        _same((ref[0].clone(), ref[1]), (got[0].clone(), got[1]), "precond seed %d" % seed)
        p.close()


@pytest.mark.parametrize("kind", ["uno", "jacobi"])
def test_graph_mode_elastic(orc, uno, kind):
    shape = (12, 10, 9)
    ph, _ = si.rsa_inclusions(shape, 2, 4, 0.3, 77)
    lam, mu = orc.lame(si.two_phase_kappa(ph, 1.0, 100.0), 0.3)
    P = None
    if kind == "uno":
        M = 3
        rng = np.random.default_rng(78)
        th = 0.3 * rng.standard_normal(orc.num_weights3(M))
        th.reshape(-1, 6)[:, [0, 1, 3]] += 1.0
        P = uno.UnoPrecond.create_elastic(shape, M, th)
    loads = np.eye(6)
    kw = dict(kind=kind, precond=P, rtol=1e-9)
    ua, ia = uno.el_pcg_solve(T(lam), T(mu), loads, **kw)
    ua = ua.clone()
    for rep in range(2):
        ub, ib = uno.el_pcg_solve(T(lam), T(mu), loads, use_graphs=True, **kw)
        _same((ua, ia), (ub, ib), "elastic %s rep %d" % (kind, rep))


def test_graph_mode_many_problems(uno):
    shapes = [(48, 40), (24, 24, 24), (20, 16, 12), (48, 40), (24, 24, 24)]
    precs = {s: _precond(uno, s, 3, 80 + i) for i, s in enumerate(sorted(set(shapes)))}
    probs = []
    for i, s in enumerate(shapes):
        probs.append(dict(kappa=T(_kappa(s, 90 + i)), loads=np.eye(len(s)), precond=precs[s]))

    def run(graphs):
        for P in probs:
            P.pop("u", None)
        us, infos = uno.pcg_solve_many(probs, kind="uno", rtol=1e-9, use_graphs=graphs)
        return [u.clone() for u in us], infos

    ua, ia = run(False)
    for rep in range(2):
        ub, ib = run(True)
        for j in range(len(shapes)):
            assert [x["iters"] for x in ia[j]] == [x["iters"] for x in ib[j]]
            assert torch.equal(ua[j], ub[j]), "problem %d rep %d" % (j, rep)
