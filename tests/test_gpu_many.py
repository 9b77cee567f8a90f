"""GPU: many problems of uneven sizes in one call (2D and 3D grids mixed,
1-3 load cases each, Jacobi-CG and UNO-CG): every load case equals the
oracle's solution, and equals the same problem solved on its own."""
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


SHAPES = [(12, 12), (16, 20), (8, 8, 8), (10, 12, 8), (12, 12)]


def work_list(seed):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(11):
        shape = SHAPES[i % len(SHAPES)]
        ph, _ = si.rsa_inclusions(shape, 1.5, 2.5, 0.25, seed + i)
        contrast = float(np.exp(rng.uniform(np.log(10.0), np.log(1000.0))))
        kap = si.two_phase_kappa(ph, 1.0, contrast)
        nl = 1 + i % 3 if len(shape) == 3 else 1 + i % 2
        loads = rng.standard_normal((nl, len(shape)))
        probs.append((kap, loads))
    return probs


def test_many_jacobi_matches_oracle_and_single(orc, uno):
    probs = work_list(300)
    us, infos = uno.pcg_solve_many([{"kappa": T(k), "loads": l} for k, l in probs], kind="jacobi", rtol=1e-10)
    for (kap, loads), u, inf in zip(probs, us, infos):
        assert len(inf) == len(loads)
        ub, ib = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="jacobi", rtol=1e-10)
        for j in range(len(loads)):
            assert inf[j]["converged"]
            uo, ito, _, _ = orc.pcg(kap, orc.rhs(kap, loads[j]), "jacobi", rtol=1e-10)
            ug = u[j].cpu().numpy()
            assert np.abs(ug - uo).max() < 1e-8 * np.abs(uo).max()
            assert abs(inf[j]["iters"] - ito) <= max(1, int(0.03 * ito))
            assert (u[j] - ub[j]).abs().max().item() < 1e-8 * ub[j].abs().max().item()


def test_many_uno_per_grid_preconditioners(orc, uno):
    probs = work_list(400)
    pre = {}
    for kap, _ in probs:
        shape = kap.shape
        if shape not in pre:
            M = 2
            pre[shape] = uno.UnoPrecond.create(shape, M, si.random_theta(uno.num_weights(len(shape), M), 7,
                                                                         scale=0.05))
    us, infos = uno.pcg_solve_many([{"kappa": T(k), "loads": l, "precond": pre[k.shape]} for k, l in probs],
                                   kind="uno", rtol=1e-9)
    for (kap, loads), u, inf in zip(probs, us, infos):
        P = pre[kap.shape]
        ub, ib = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="uno", precond=P, rtol=1e-9)
        for j in range(len(loads)):
            assert inf[j]["converged"]
            assert abs(inf[j]["iters"] - ib[j]["iters"]) <= 1
            scale = ub[j].abs().max().item()
            assert (u[j] - ub[j]).abs().max().item() < 1e-7 * scale


def test_many_errors_and_empty(uno):
    assert uno.pcg_solve_many([], kind="jacobi") == ([], [])
    k = T(np.ones((8, 8)))
    with pytest.raises(uno.UnoError):
        uno.pcg_solve_many([{"kappa": k, "loads": np.zeros((4, 2))}], kind="jacobi")  # 4 loads
    with pytest.raises(uno.UnoError):
        uno.pcg_solve_many([{"kappa": k, "loads": np.eye(2)}], kind="uno")  # no preconditioner


def test_many_fp32_mode_matches_fp64(orc, uno):
    """FP32 operator and preconditioner with FP64 reductions over the whole
    work list: every effective tensor within 1e-5 of the FP64 one."""
    probs = work_list(500)
    pre = {}
    for kap, _ in probs:
        if kap.shape not in pre:
            # M = 1: the learned-mode passes (which the FP32 mode needs) exist on every grid here
            pre[kap.shape] = uno.UnoPrecond.create(kap.shape, 1, si.random_theta(uno.num_weights(len(kap.shape), 1),
                                                                                7, scale=0.05))
    items = [{"kappa": T(k), "loads": l, "precond": pre[k.shape]} for k, l in probs]
    u64, i64 = uno.pcg_solve_many(items, kind="uno", rtol=1e-8)
    items = [{"kappa": T(k), "loads": l, "precond": pre[k.shape]} for k, l in probs]
    u32, i32 = uno.pcg_solve_many(items, kind="uno", rtol=1e-8, op_dtype=torch.float32, prec_dtype=torch.float32)
    for (kap, loads), a, b, ia, ib in zip(probs, u64, u32, i64, i32):
        assert all(i["converged"] for i in ia + ib)
        assert all(i["true_rel_res"] <= 1e-8 * (1 + 1e-6) for i in ia + ib)
        d = len(kap.shape)
        if len(loads) == d:
            ka = uno.effective_tensor(T(kap), loads, a)
            kb = uno.effective_tensor(T(kap), loads, b)
            assert np.abs(kb - ka).max() < 1e-5 * np.abs(ka).max()
        assert (a - b).abs().max().item() < 1e-4 * a.abs().max().item()


def test_many_bf16_mode_matches_fp64(uno):
    """The BF16 preconditioner storage mode over the whole work list (FP32
    operator; the learned-mode passes' table and spectrum in BF16): every
    solve reaches its tolerance with its true FP64 residual, and every
    effective tensor is within 1e-5 of the FP64 one."""
    probs = work_list(500)
    pre = {}
    for kap, _ in probs:
        if kap.shape not in pre:
            pre[kap.shape] = uno.UnoPrecond.create(kap.shape, 1, si.random_theta(uno.num_weights(len(kap.shape), 1),
                                                                                7, scale=0.05))
    items = [{"kappa": T(k), "loads": l, "precond": pre[k.shape]} for k, l in probs]
    u64, i64 = uno.pcg_solve_many(items, kind="uno", rtol=1e-8)
    items = [{"kappa": T(k), "loads": l, "precond": pre[k.shape]} for k, l in probs]
    u16, i16 = uno.pcg_solve_many(items, kind="uno", rtol=1e-8, op_dtype=torch.float32, prec_dtype=torch.bfloat16)
    for (kap, loads), a, b, ia, ib in zip(probs, u64, u16, i64, i16):
        assert all(i["converged"] for i in ia + ib)
        assert all(i["true_rel_res"] <= 1e-8 * (1 + 1e-6) for i in ia + ib)
        d = len(kap.shape)
        if len(loads) == d:
            ka = uno.effective_tensor(T(kap), loads, a)
            kb = uno.effective_tensor(T(kap), loads, b)
            assert np.abs(kb - ka).max() < 1e-5 * np.abs(ka).max()


@pytest.mark.parametrize("kind", ["jacobi", "uno"])
def test_many_fp32_mode_true_residual_at_exit(uno, kind):
    """FP32 mode on larger high-contrast cells (2D 256^2 and 128^2, 3D 32^3,
    contrast 1000, rel. residual 1e-6): the recursive residual of the last
    restart cycle drifts from f - A u by the FP32 operator's rounding, and the
    exit check in FP64 reopens such loads, so every load ends with its true
    residual within the tolerance."""
    items = []
    for j, shape in enumerate([(256, 256), (128, 128), (32, 32, 32), (256, 256)]):
        d = len(shape)
        ph, _ = si.rsa_inclusions(shape, shape[0] / 16.0, shape[0] / 8.0, 0.25, 900 + j)
        it = {"kappa": T(si.two_phase_kappa(ph, 1.0, 1000.0)), "loads": np.eye(d)}
        if kind == "uno":
            it["precond"] = uno.UnoPrecond.create(shape, 4, si.random_theta(uno.num_weights(d, 4), 11 + j,
                                                                            scale=0.05))
        items.append(it)
    _, infos = uno.pcg_solve_many(items, kind=kind, rtol=1e-6, max_iter=50000, op_dtype=torch.float32,
                                  prec_dtype=torch.float32)
    for inf in infos:
        for i in inf:
            assert i["converged"], i
            assert i["true_rel_res"] <= 1e-6 * (1 + 1e-6), i
