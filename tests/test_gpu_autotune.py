"""GPU: the operator autotuner records a shape the later solves use, and
solves with the recorded shape still match the oracle (the shape changes
only how the d.Ad partial sums are grouped).  Grids of their own, so that
no other test's shapes are affected by the records."""
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


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def _kappa(shape, seed):
    ph, _ = si.rsa_inclusions(shape, 2, 4, 0.25, seed)
    return si.two_phase_kappa(ph, 1.0, 100.0)


def test_autotune_shared_field_then_solve(orc, uno):
    shape = (26, 22, 18)
    kap = _kappa(shape, 61)
    loads = np.eye(3)
    before, ib = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="jacobi", rtol=1e-12)
    rec = uno.autotune_operator(shape, 3, kappa_per_rhs=False)
    print("autotuned", shape, rec, flush=True)
    assert rec["tz"] in (16, 32, 64) and rec["ry"] in (1, 2) and 2 <= rec["xb"] <= shape[0] and rec["us"] > 0
    after, ia = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="jacobi", rtol=1e-12)
    for j, g in enumerate(loads):
        uo, _, _, _ = orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-12)
        assert rel(after[j].cpu().numpy(), uo) < 1e-8
        assert abs(ia[j]["iters"] - ib[j]["iters"]) <= 1
    # FP32 records are kept apart from FP64 ones
    rec32 = uno.autotune_operator(shape, 3, dtype=torch.float32)
    assert rec32["tz"] in (16, 32, 64)


def test_autotune_per_rhs_fields_batch(uno):
    shape = (48, 48, 48)
    n = 8
    kaps = T(np.stack([_kappa(shape, 70 + i) for i in range(n)]))
    loads = np.tile(np.eye(3)[0], (n, 1))
    th = si.random_theta(uno.num_weights(3, 4), 3, scale=0.05, spread=0.2)
    p = uno.UnoPrecond.create(shape, 4, th)
    ref, ir = uno.pcg_solve_batch(kaps, macro_loads=loads, kind="uno", precond=p, rtol=1e-10, kappa_per_rhs=True)
    ref = ref.clone()
    rec = uno.autotune_operator(shape, n, kappa_per_rhs=True)
    print("autotuned", shape, n, rec, flush=True)
    got, ig = uno.pcg_solve_batch(kaps, macro_loads=loads, kind="uno", precond=p, rtol=1e-10, kappa_per_rhs=True)
    # random weights make a poor preconditioner (about 700 passes), where the
    # regrouped d.Ad sums move the count by a few passes per hundred
    for a, b in zip(ir, ig):
        assert b["converged"] and abs(a["iters"] - b["iters"]) <= max(1, int(0.03 * a["iters"]))
    assert rel(got.cpu().numpy(), ref.cpu().numpy()) < 1e-8


MARCH_SHAPES = [(64, 1), (32, 1), (16, 1), (64, 2), (32, 2)]


@pytest.mark.parametrize("tz,ry", MARCH_SHAPES)
def test_every_march_shape_matches_oracle(orc, uno, tz, ry):
    """Each built footprint (tz, ry), pinned through set_operator_shape, on a
    grid ragged along y and z (37 rows, 70 = 64 + 6 columns) and with
    several plane counts per workgroup: the apply equals the oracle's."""
    shape = (13, 37, 70)
    print("march shape", tz, ry, flush=True)
    kap = si.random_field(shape, 81, 0.1, 10.0)
    u = si.random_field(shape, 82)
    ref = orc.fe_apply(kap, u)
    for xb in (2, 5, 13):
        uno.set_operator_shape(shape, 1, tz, ry, xb)
        y = uno.fe_apply(T(kap), T(u)).cpu().numpy()
        assert rel(y, ref) < 1e-12, (tz, ry, xb)
        uno.set_operator_shape(shape, 1, tz, ry, xb, dtype=torch.float32)
        y32 = uno.fe_apply(torch.tensor(kap, dtype=torch.float32, device=DEV),
                           torch.tensor(u, dtype=torch.float32, device=DEV)).cpu().numpy()
        ref32 = orc.fe_apply(kap.astype(np.float32), u.astype(np.float32))
        assert rel(y32, ref32) < 1e-5, (tz, ry, xb)


@pytest.mark.parametrize("tz,ry", [(64, 2), (32, 2)])
def test_two_row_march_inside_cg_matches_oracle(orc, uno, tz, ry):
    """The two-row footprints inside batched CG (the fused direction update,
    d.p partials) on a grid smaller than the 64-wide footprint along z:
    solutions equal the oracle's to the solve tolerance."""
    shape = (16, 24, 40)
    kap = _kappa(shape, 83)
    loads = np.eye(3)
    uno.set_operator_shape(shape, 3, tz, ry, 3)
    got, info = uno.pcg_solve_batch(T(kap), macro_loads=loads, kind="jacobi", rtol=1e-12)
    for j, g in enumerate(loads):
        uo, its, _, _ = orc.pcg(kap, orc.rhs(kap, g), "jacobi", rtol=1e-12)
        assert info[j]["converged"]
        assert rel(got[j].cpu().numpy(), uo) < 1e-8
        assert abs(info[j]["iters"] - its) <= max(1, int(0.01 * its))
