#!/usr/bin/env python3
"""Benchmark: UNO-CG vs Jacobi-CG on 3D 64^3 periodic thermal RVEs, one GPU.

Workload: trilinear hex8 FE on a 64^3 periodic voxel grid, two phases
(non-overlapping random spheres, radius 4-8 voxels, volume fraction 0.25,
conductivity 100 in a matrix of conductivity 1), three unit macroscopic
gradient load cases per microstructure, relative residual 1e-6 in the
infinity norm.  Synthetic seeded microstructures stand in for the paper's
voxel datasets.

One step = the whole hot path over the 16 test microstructures: the rhs
and the UNO-CG solve (operator apply, UNO preconditioner apply, CG
recurrences) to 1e-6 of their 48 load cases, carried together by every
pass kernel, then the 16 effective 3x3 conductivities.  Inputs are
resident in device memory before the timed region.  The UNO weights are
trained beforehand (untimed) on solver-generated pairs: seeded random
weights -> UNO-CG solves of training microstructures -> closed-form fit
-> more solves -> refit.

Prints one JSON line; `value` is UNO-CG FP64 DOF*iterations/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPE = (64, 64, 64)
LOADS = np.eye(3)
RTOL = 1e-6
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# this benchmark (64^3, M = 12, 48 right-hand sides per launch; the mean over
# the launches, loads that have converged returning at once), each scaled by
# what the counter reads for a device copy of known size (FETCH x 2,
# WRITE x 1); the summary with its commands is
# profiles/uno_cg_64cubed_hbm_counters.md.  Valid only for the kernel sources
# as they were when counted (TRAFFIC_SRC: hash of the files in TRAFFIC_FILES);
# after any change the figure is withheld.
TRAFFIC_FILES = ["lowrank.hip", "stencil_tile.h", "cg_ctl.h", "reduce.h", "cg.hip"]
TRAFFIC_SRC = "48d84dfe24e0c97a"
TRAFFIC_BYTES = {  # per launch of the benchmark step (48 right-hand sides)
    "k_stencil_march<double,CG>": 517589690,
    "k_lr_fwd<update,double>": 577204109,
    "k_lr_mid": 46915876,
    "k_lr_inv_pairs<double>": 235908107,
}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_FILES:
        with open(os.path.join(ROOT, "paper_2508_02681_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_families(uno, shape, M, learned, kappa_per_rhs):
    """Kernel families of one UNO-CG pass and their algorithmic bytes
    (FP64) as (per right-hand side that is still running, per launch): a
    launch carries the right-hand sides of a batch, each with its own
    conductivity field or all with one; the table is shared, and a load
    that has converged returns at once from the kernels of later passes."""
    n = int(np.prod(shape))
    kap_rhs, kap_launch = (n * 8, 0) if kappa_per_rhs else (0, n * 8)
    nspec = shape[0] * shape[1] * (shape[2] // 2 + 1)
    nblk = shape[0] * (2 * M + 1) * (M + 1)   # learned block after the two partial DFTs (y, z)
    if learned:
        # pass B -> pass C -> operator -> [update + pass A]
        fams = {uno.KT_MATVEC: "k_stencil_march<double,CG>", uno.KT_UPDATE: "k_lr_fwd<update,double>",
                uno.KT_FFT_MID: "k_lr_mid", uno.KT_FFT_INV: "k_lr_inv_pairs<double>"}
        bytes_per = {
            uno.KT_MATVEC: (n * 8 * 4 + kap_rhs, kap_launch),  # read s, d_old, kappa; write d_new, p
            uno.KT_UPDATE: (n * 8 * 6 + nblk * 16, 0),        # read r, u, d, p; write r, u, block spectrum
            uno.KT_FFT_MID: (nblk * 16 * 2, nblk * 8),        # block spectrum in/out; table
            uno.KT_FFT_INV: (n * 8 * 2 + nblk * 16, 0),       # read r, H; write s
        }
    else:  # spectral passes, one load per launch
        fams = {uno.KT_MATVEC: "k_stencil_march<double,CG>", uno.KT_UPDATE: "k_cg_update<double>",
                uno.KT_FFT_FWD: "k_fft_r2c_z", uno.KT_FFT_MID: "k_fft_strided(mid)", uno.KT_FFT_INV: "k_fft_c2r_z"}
        bytes_per = {
            uno.KT_MATVEC: (n * 8 * 5, 0),
            uno.KT_UPDATE: (n * 8 * 6, 0),               # read r, p, u, d; write r, u
            uno.KT_FFT_FWD: (n * 8 + nspec * 16, 0),     # read r; write half spectrum
            uno.KT_FFT_MID: (nspec * 16 * 2 + nspec * 8, 0),  # spectrum in/out + table
            uno.KT_FFT_INV: (nspec * 16 + n * 8 * 2, 0),  # spectrum in; write s; read r (r.s)
        }
    return fams, bytes_per


def family_times(uno, fams, run):
    """Summed duration (ms) and launch count of each kernel family over one
    call of run(), from start/stop events of the launches themselves, and
    the passes of each right-hand side in that run (run() returns them)."""
    import torch
    out = {}
    passes = None
    for fam in fams:
        uno.timing_enable(fam)
        passes = run()
        torch.cuda.synchronize()
        out[fam] = uno.timing_read()
        uno.timing_enable(uno.KT_NONE)
    return out, passes


def roofline_record(fams, bytes_per, timed):
    """Dominant family (largest total time): achieved = algorithmic bytes
    of the run / its summed launch time, the bytes counting each right-hand
    side for the passes it ran (sum of passes x per-load bytes) plus the
    per-launch part; bytes_per_launch is that total over the launches."""
    fam_ms, passes = timed
    tot_passes = float(sum(passes))
    def total_bytes(f):
        per_rhs, per_launch = bytes_per[f]
        return tot_passes * per_rhs + fam_ms[f][1] * per_launch
    dom = max(fam_ms, key=lambda f: fam_ms[f][0])
    tot, nl = fam_ms[dom]
    avg_s = tot / max(nl, 1) / 1e3
    bpl = total_bytes(dom) / max(nl, 1)
    achieved = bpl / avg_s / 1e9
    per_us = {fams[f]: fam_ms[f][0] / max(fam_ms[f][1], 1) * 1e3 for f in fams}
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": fams[dom], "avg_us": round(avg_s * 1e6, 2), "bytes_per_launch": round(bpl),
            "per_family_us": {k: round(v, 2) for k, v in per_us.items()},
            "per_family_GBs": {fams[f]: round(total_bytes(f) / max(fam_ms[f][0], 1e-9) / 1e6, 1) for f in fams},
            "per_family_ms_per_run": {fams[f]: round(fam_ms[f][0], 3) for f in fams},
            "per_family_launches": {fams[f]: int(fam_ms[f][1]) for f in fams}}


def elastic_families(uno, shape, M):
    """Kernel families of one elastic UNO-CG pass (c = 3, planar components,
    one Lame field pair for all right-hand sides) and their algorithmic
    bytes as (per running right-hand side, per launch)."""
    n = int(np.prod(shape))
    nblk = 3 * shape[0] * (2 * M + 1) * (M + 1)  # learned block of the three components after pass A
    fams = {uno.KT_MATVEC: "k_el_march<CG>", uno.KT_UPDATE: "k_lr_fwd<update,double>(c=3)",
            uno.KT_FFT_MID: "k_lr_mid3", uno.KT_FFT_INV: "k_lr_inv<double,c=3>"}
    bytes_per = {
        uno.KT_MATVEC: (3 * n * 8 * 4, 2 * n * 8),    # read s, d_old; write d_new, p; lambda, mu
        uno.KT_UPDATE: (3 * n * 8 * 6 + nblk * 16, 0),  # read r, u, d, p; write r, u, block spectrum
        uno.KT_FFT_MID: (nblk * 16 * 2, nblk // 3 * 48),  # block spectrum in/out; 6 table entries
        uno.KT_FFT_INV: (3 * n * 8 * 2 + nblk * 16, 0),  # read r, H; write s
    }
    return fams, bytes_per


def elastic_record(uno, si, torch, dev, M):
    """3D linear elasticity, 128^3, six Mandel loads: UNO-CG (trained on
    Jacobi-CG solutions of two other microstructures) in FP64 and in the FP32
    mode vs Jacobi-CG FP64, relative residual 1e-6, effective 6 x 6
    stiffness."""
    cfg = dict(si.CONFIG_EL_128)
    shape = cfg["shape"]
    n = int(np.prod(shape))
    loads = np.eye(6)

    def lame(seed):
        E, frac = si.microstructure(cfg, seed)
        nu = cfg["nu"]
        return (torch.tensor(E * nu / ((1 + nu) * (1 - 2 * nu)), device=dev),
                torch.tensor(E / (2 * (1 + nu)), device=dev), frac)

    t0 = time.time()
    fs, us = [], []
    for seed in cfg["train_seeds"]:
        L, Mu, _ = lame(seed)
        u, _ = uno.el_pcg_solve(L, Mu, loads, rtol=1e-8)
        fs += [uno.el_macro_rhs(L, Mu, loads[j]) for j in range(6)]
        us += [u[j].clone() for j in range(6)]
    nh = shape[2] // 2 + 1
    A = torch.zeros((6, shape[0], shape[1], nh), dtype=torch.float64, device=dev)
    B = torch.zeros_like(A)
    uno.el_uno_train_accumulate(torch.stack(fs), torch.stack(us), A, B, len(fs))
    th, _ = uno.el_uno_train_fit(shape, M, A, B)
    P = uno.UnoPrecond.create_elastic(shape, M, th)
    del fs, us, A, B
    log("elastic 128^3: trained M = %d on %d pairs in %.1fs" % (M, 6 * len(cfg["train_seeds"]), time.time() - t0))
    L, Mu, frac = lame(cfg["test_seeds"][0])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(**kw):
        uno.el_pcg_solve(L, Mu, loads, rtol=RTOL, max_iter=3, **kw)  # warm-up: workspace, plans
        torch.cuda.synchronize()
        ev0.record()
        u, inf = uno.el_pcg_solve(L, Mu, loads, rtol=RTOL, **kw)
        ev1.record()
        torch.cuda.synchronize()
        return u, inf, ev0.elapsed_time(ev1)

    uu, iu, tu = timed(kind="uno", precond=P)
    uj, ij, tj = timed(kind="jacobi")
    u32, i32, t32 = timed(kind="uno", precond=P, op_dtype=torch.float32)
    Du = uno.el_effective_stiffness(L, Mu, loads, uu)
    Dj = uno.el_effective_stiffness(L, Mu, loads, uj)
    D32 = uno.el_effective_stiffness(L, Mu, loads, u32)
    del u32
    fams, bytes_per = elastic_families(uno, shape, M)

    def run():
        return [i["iters"] for i in uno.el_pcg_solve(L, Mu, loads, kind="uno", precond=P, rtol=RTOL)[1]]

    rec = roofline_record(fams, bytes_per, family_times(uno, fams, run))
    its_u = [i["iters"] for i in iu]
    its_j = [i["iters"] for i in ij]
    out = {
        "workload": "3D elasticity 128^3 periodic hex8 (3 DOF/node, 6.3M DOF), spheres r 8-16 vf %.2f, E 1/100, "
                    "nu 0.3, 6 Mandel strain loads solved together, rel. residual 1e-6, FP64" % frac,
        "M": M,
        "uno_cg": {"passes": its_u, "ms_per_solve": tu / 6, "converged": all(i["converged"] for i in iu),
                   "dof_iters_per_s": 3 * n * sum(its_u) / (tu * 1e-3)},
        "jac_cg": {"passes": its_j, "ms_per_solve": tj / 6, "converged": all(i["converged"] for i in ij),
                   "dof_iters_per_s": 3 * n * sum(its_j) / (tj * 1e-3)},
        "uno_cg_fp32": {"passes": [i["iters"] for i in i32], "ms_per_solve": t32 / 6,
                        "converged": all(i["converged"] for i in i32),
                        "stiffness_rel_diff_vs_fp64_jac_cg": float(np.abs(D32 - Dj).max() / np.abs(Dj).max()),
                        "note": "FP32 operator, preconditioner and direction; FP64 residuals, reductions, stop test"},
        "time_to_tol_speedup_uno_vs_jac": tj / tu,
        "time_to_tol_speedup_uno_fp32_vs_jac_fp64": tj / t32,
        "true_rel_res_max": {"uno_cg": max(i["true_rel_res"] for i in iu),
                             "jac_cg": max(i["true_rel_res"] for i in ij),
                             "uno_cg_fp32": max(i["true_rel_res"] for i in i32)},
        "stiffness_uno": np.round(Du, 6).tolist(),
        "stiffness_rel_diff_uno_vs_jac": float(np.abs(Du - Dj).max() / np.abs(Dj).max()),
        "per_kernel": {k: rec[k] for k in ("kernel", "avg_us", "per_family_us", "per_family_GBs", "per_family_ms_per_run",
                                           "per_family_launches")},
    }
    log("elastic 128^3: UNO-CG %.1f ms/solve (%d passes), Jac-CG %.1f ms/solve (%d passes), speedup %.2f; "
        "UNO-CG FP32 %.1f ms/solve (%d passes), stiffness vs FP64 %.1e" %
        (tu / 6, max(its_u), tj / 6, max(its_j), tj / tu, t32 / 6, max(i["iters"] for i in i32),
         out["uno_cg_fp32"]["stiffness_rel_diff_vs_fp64_jac_cg"]))
    log("elastic 128^3 per kernel: " + ", ".join("%s %.0f us %.0f GB/s" % (k, rec["per_family_us"][k], v)
                                                  for k, v in rec["per_family_GBs"].items()))
    return out


TUNED_192 = {}


def tune_192(uno, tune=True):
    """The project's autotuner for the operator march at 192^3 (one shared
    conductivity field, one and three right-hand sides per launch), once per
    process: the records are used by every later solve and apply of those
    launch shapes (UNO-CG and Jacobi-CG alike)."""
    if tune and not TUNED_192:
        for nr in (1, 3):
            TUNED_192[nr] = uno.autotune_operator((192, 192, 192), nr)
        log("autotuned operator march (192^3): %s" % TUNED_192)
    return dict(TUNED_192)


def paper192_record(uno, si, torch, dev, tune=True):
    """The paper's 3D thermal size and contrast (192^3, R = 5, synthetic
    spheres standing in for its dataset): UNO-CG (trained untimed on the
    Jacobi-CG solutions of four other microstructures, M picked on a fifth)
    and Jacobi-CG to 1e-6, FP64, one load alone and the three loads
    together.  Context next to the paper's published timings on other
    hardware, not the headline."""
    cfg = dict(si.CONFIG_3D_192_R5)
    shape = cfg["shape"]
    tuned = tune_192(uno, tune)
    n = int(np.prod(shape))
    loads = np.eye(3)
    t0 = time.time()
    hs = uno.half_shape(shape)
    A = torch.zeros(hs, dtype=torch.float64, device=dev)
    B = torch.zeros_like(A)
    for seed in cfg["train_seeds"]:
        kt = torch.tensor(si.microstructure(cfg, seed)[0], device=dev)
        u2, _ = uno.pcg_solve_batch(kt, macro_loads=loads, kind="jacobi", rtol=1e-8, max_iter=50000)
        F = torch.stack([uno.uno_macro_rhs(kt, loads[a]) for a in range(3)])
        uno.uno_train_accumulate(F, u2, A, B, 3 * len(cfg["train_seeds"]))
        del u2, F
    kv = torch.tensor(si.microstructure(cfg, cfg["val_seed"])[0], device=dev)
    best = None
    for M in (8, 12, 16):
        P = uno.UnoPrecond.create(shape, M, uno.uno_train_fit(shape, M, A, B))
        uno.pcg_solve_batch(kv, macro_loads=loads, kind="uno", precond=P, rtol=RTOL)
        torch.cuda.synchronize()
        t = time.perf_counter()
        uno.pcg_solve_batch(kv, macro_loads=loads, kind="uno", precond=P, rtol=RTOL)
        torch.cuda.synchronize()
        tv = time.perf_counter() - t
        if best is None or tv < best[0]:
            best = (tv, M, P)
    _, M, P = best
    del A, B, kv
    log("192^3 R = 5: trained on %d pairs, M = %d picked, in %.1fs" % (3 * len(cfg["train_seeds"]), M, time.time() - t0))
    kt = torch.tensor(si.microstructure(cfg, cfg["test_seed"])[0], device=dev)

    def timed(kind, precond, all_loads):
        kw = dict(kind=kind, precond=precond, rtol=RTOL, max_iter=50000)
        if all_loads:
            f = lambda: uno.pcg_solve_batch(kt, macro_loads=loads, **kw)[1]
        else:
            f = lambda: [uno.pcg_solve(kt, macro_load=loads[0], **kw)[1]]
        f()
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, infos

    out = {"workload": "3D thermal 192^3 (%d DOF), spheres r 12-24 vf 0.25, kappa 1 / 0.2 (R = 5), FP64 to 1e-6; "
                       "the paper's size and contrast with synthetic microstructures" % n, "M": M,
           "operator_shape_autotuned": tuned}
    for kind, pc in (("uno_cg", P), ("jac_cg", None)):
        t1, i1 = timed("uno" if pc else "jacobi", pc, False)
        t3, i3 = timed("uno" if pc else "jacobi", pc, True)
        out[kind] = {"ms_one_load": t1, "passes_one_load": i1[0]["iters"], "ms_per_solve_3_loads_together": t3 / 3,
                     "passes_3_loads": [i["iters"] for i in i3],
                     "true_rel_res_max": max(i["true_rel_res"] for i in i1 + i3)}
    out["time_to_tol_ratio_one_load"] = out["jac_cg"]["ms_one_load"] / out["uno_cg"]["ms_one_load"]
    log("192^3 R = 5: UNO-CG %.1f ms (%d passes) one load, Jac-CG %.1f ms (%d passes), ratio %.1f" %
        (out["uno_cg"]["ms_one_load"], out["uno_cg"]["passes_one_load"], out["jac_cg"]["ms_one_load"],
         out["jac_cg"]["passes_one_load"], out["time_to_tol_ratio_one_load"]))
    return out


def many_record(uno, si, torch, dev):
    """Many-query workload: 256 problems of uneven sizes (2D 64^2/128^2/256^2,
    3D 32^3/48^3), contrast log-uniform in [10, 1000], 2 or 3 loads each,
    UNO-CG FP64 to 1e-6 with one trained preconditioner per grid size, all
    in one pcg_solve_many call; against the same problems one at a time and
    against Jacobi-CG in one call."""
    cfg = dict(si.CONFIG_MANY)
    t0 = time.time()
    probs = [si.many_problem(cfg, i) for i in range(cfg["count"])]
    kaps = [torch.tensor(k, device=dev) for k, _ in probs]
    Ms = {2: {64: 8, 128: 12, 256: 16}, 3: {32: 6, 48: 8}}
    pre = {}
    for shape in cfg["shapes"]:  # train one preconditioner per size on pairs of extra problems
        d = len(shape)
        hs = uno.half_shape(shape)
        A = torch.zeros(hs, dtype=torch.float64, device=dev)
        B = torch.zeros_like(A)
        nt = cfg["train_per_shape"]
        rng = np.random.default_rng(cfg["seed"] + 100000 + shape[0] * d)
        for j in range(nt):  # training cells of this size, contrasts over the same range
            ph, _ = si.rsa_inclusions(shape, shape[0] / 16.0, shape[0] / 8.0, cfg["vf"],
                                      cfg["seed"] + 200000 + 1000 * shape[0] + 10 * d + j)
            contrast = float(np.exp(rng.uniform(np.log(cfg["contrast"][0]), np.log(cfg["contrast"][1]))))
            kt = torch.tensor(si.two_phase_kappa(ph, 1.0, contrast), device=dev)
            loads = np.eye(d)
            u, _ = uno.pcg_solve_batch(kt, macro_loads=loads, kind="jacobi", rtol=1e-8)
            F = torch.stack([uno.uno_macro_rhs(kt, loads[a]) for a in range(d)])
            uno.uno_train_accumulate(F, u, A, B, nt * d)
        M = Ms[d][shape[0]]
        pre[shape] = uno.UnoPrecond.create(shape, M, uno.uno_train_fit(shape, M, A, B))
    log("many: %d problems generated, %d preconditioners trained in %.1fs" % (len(probs), len(pre), time.time() - t0))
    items = [{"kappa": kt, "loads": l, "precond": pre[tuple(kt.shape)]} for kt, (_, l) in zip(kaps, probs)]
    nsolve = sum(len(l) for _, l in probs)
    dofs = [int(np.prod(kt.shape)) for kt in kaps]
    worst = {}  # largest true relative residual at exit (FP64), per run

    def run_many(kind, **kw):
        for it in items:
            it["u"] = torch.zeros((len(it["loads"]),) + tuple(it["kappa"].shape), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        us, infos = uno.pcg_solve_many(items, kind=kind, rtol=RTOL, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        dit = sum(n * sum(i["iters"] for i in inf) for n, inf in zip(dofs, infos))
        conv = all(i["converged"] for inf in infos for i in inf)
        tag = kind + ("_fp32" if kw.get("op_dtype") is not None else "") + ("_graphs" if kw.get("use_graphs") else "")
        worst[tag] = max(i["true_rel_res"] for inf in infos for i in inf)
        return dt, dit, conv, us

    run_many("uno")  # warm-up: workspaces, streams
    dt, dit, conv, us = run_many("uno")
    dtj, ditj, convj, _ = run_many("jacobi")
    f32 = dict(op_dtype=torch.float32, prec_dtype=torch.float32)
    run_many("uno", **f32)
    dtm, ditm, convm, _ = run_many("uno", **f32)
    run_many("uno", use_graphs=True)  # warm-up: captured chunks
    dtg, ditg, convg, _ = run_many("uno", use_graphs=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for it in items:
        uno.pcg_solve_batch(it["kappa"], macro_loads=it["loads"], kind="uno", precond=it["precond"], rtol=RTOL)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t
    out = {
        "workload": "%d problems: 2D 64^2/128^2/256^2 and 3D 32^3/48^3 (drawn uniformly), spheres/discs r N/16-N/8 "
                    "vf 0.25, contrast log-uniform [10, 1000], %d solves (2 loads in 2D, 3 in 3D), UNO-CG FP64 to 1e-6, "
                    "one trained preconditioner per size" % (len(probs), nsolve),
        "solves": nsolve,
        "uno_cg_many": {"s": dt, "solves_per_s": nsolve / dt, "dof_iters_per_s": dit / dt, "converged": conv},
        "jac_cg_many": {"s": dtj, "solves_per_s": nsolve / dtj, "dof_iters_per_s": ditj / dtj, "converged": convj},
        "uno_cg_many_fp32": {"s": dtm, "solves_per_s": nsolve / dtm, "dof_iters_per_s": ditm / dtm,
                             "converged": convm, "note": "FP32 operator and preconditioner, FP64 reductions"},
        "uno_cg_many_graphs": {"s": dtg, "solves_per_s": nsolve / dtg, "dof_iters_per_s": ditg / dtg,
                               "converged": convg, "note": "passes replayed from captured hipGraphs of 8 passes"},
        "uno_cg_one_problem_at_a_time": {"s": dts, "solves_per_s": nsolve / dts},
        "speedup_many_vs_one_at_a_time": dts / dt,
        "true_rel_res_max": worst,
        "time_to_tol_speedup_uno_vs_jac": dtj / dt,
    }
    log("many: UNO-CG %.3f s (%.0f solves/s), graphs %.3f s, FP32 %.3f s, one at a time %.3f s, Jacobi-CG %.3f s" %
        (dt, nsolve / dt, dtg, dtm, dts, dtj))
    return out


def oracle_kbar_errors(kap, results):
    """Relative difference (max entry / max entry) of each GPU kappa_bar of
    one microstructure against the FP64 oracle's (Jacobi-CG to rtol 1e-10
    for each load, the three loads in worker processes at once)."""
    import multiprocessing as mp
    import oracle
    jobs = [(kap, g, "jacobi", None, 0, 1e-10) for g in LOADS]
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        sols = pool.map(oracle.pcg_solution, jobs)
    kb_o = oracle.effective_tensor(kap, sols, list(LOADS))
    out = {"reference": "oracle Jacobi-CG (FP64) to rtol 1e-10 on test microstructure 1000, three loads",
           "oracle_s": time.perf_counter() - t, "kappa_bar_oracle": np.round(kb_o, 8).tolist()}
    for k, kb in results.items():
        out[k] = float(np.abs(np.asarray(kb) - kb_o).max() / np.abs(kb_o).max())
    log("kappa_bar vs FP64 oracle: " + ", ".join("%s %.1e" % (k, out[k]) for k in results))
    return out


def call_rooflines(uno, si, torch, dev, cfg, reps=20):
    """The two C-ABI applies the hot path is built from, each timed on its
    own at 192^3 (7.1M nodes, beyond the last-level cache): fe_apply (read
    u, kappa; write y: 24 B/node FP64, 12 FP32) and uno_precond_apply (read r,
    write s: 16 B/node, plus the learned-mode scratch; the table is 8125
    values).  HIP events around reps back-to-back calls on the stream."""
    shape = (192, 192, 192)
    n = int(np.prod(shape))
    kap = torch.tensor(si.microstructure(dict(cfg, shape=shape, r_min=12.0, r_max=24.0), 7000)[0], device=dev)
    x = torch.tensor(si.random_field(shape, 11), device=dev)
    p = uno.UnoPrecond.create(shape, 12, si.random_theta(uno.num_weights(3, 12), 12, scale=0.05, spread=0.1))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_it(fn):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e3 / reps  # us per call

    out = {"grid": list(shape), "peak_GBs": HBM_PEAK_GBS}
    y = torch.empty_like(x)
    k32, x32 = kap.float(), x.float()
    y32 = torch.empty_like(x32)
    s = torch.empty_like(x)
    recs = [("fe_apply_f64", lambda: uno.fe_apply(kap, x, y), 24 * n),
            ("fe_apply_f32", lambda: uno.fe_apply(k32, x32, y32), 12 * n),
            ("uno_precond_apply_f64", lambda: p.apply(x, s), 16 * n)]
    for name, fn, nbytes in recs:
        us = time_it(fn)
        gbs = nbytes / (us * 1e-6) / 1e9
        out[name] = {"us": round(us, 2), "alg_bytes": nbytes, "achieved_GBs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    log("192^3 calls: " + ", ".join("%s %.0f GB/s" % (k, v["achieved_GBs"]) for k, v in out.items()
                                     if isinstance(v, dict)))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_record(kaps, theta, M, n_dof, workers):
    """The oracle (FP64, one thread per solve, not tuned) on the host cores.
    One core: one full UNO-CG and one full Jacobi-CG solve to 1e-6 (test
    microstructure 1000, load e1).  All cores: one full UNO-CG solve per
    worker process (test microstructures and loads in turn), all at once;
    throughput = DOF x passes summed over the workers / wall time."""
    import multiprocessing as mp
    import oracle
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    n = max(1, min(usable, workers))
    g0 = LOADS[0]
    it_u, t_u = oracle.timed_pcg((kaps[0], g0, "uno", theta, M, RTOL))
    it_j, t_j = oracle.timed_pcg((kaps[0], g0, "jacobi", theta, M, RTOL))
    log("oracle, one core: UNO-CG %d passes in %.1f s, Jacobi-CG %d passes in %.1f s" % (it_u, t_u, it_j, t_j))
    jobs = [(kaps[i % len(kaps)], LOADS[(i // len(kaps)) % 3], "uno", theta, M, RTOL) for i in range(n)]
    ctx = mp.get_context("spawn")  # fresh interpreters: the workers never touch the GPU
    with ctx.Pool(n) as pool:
        t = time.perf_counter()  # (includes the workers' import of the oracle, well under a second)
        res = pool.map(oracle.timed_pcg, jobs, chunksize=1)
        wall = time.perf_counter() - t
    passes = sum(r[0] for r in res)
    log("oracle, %d cores: %d UNO-CG solves (%d passes) in %.1f s" % (n, n, passes, wall))
    return {"value": n_dof * passes / wall, "unit": "DOF*iters/s", "cores": n, "kind": "oracle",
            "sample": "%d oracle UNO-CG solves to 1e-6 (FP64, one process and thread each, test microstructures "
                      "and loads in turn) at once on %d cores: %d passes in %.1f s" % (n, n, passes, wall),
            "solves_per_s": n / wall,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": usable,
            "single_core": {"value": n_dof * it_u / t_u, "unit": "DOF*iters/s", "cores": 1,
                            "uno_cg_time_to_1e-6_s": t_u, "uno_cg_passes": it_u,
                            "jac_cg_time_to_1e-6_s": t_j, "jac_cg_passes": it_j,
                            "jac_cg_dof_iters_per_s": n_dof * it_j / t_j,
                            "sample": "one full oracle UNO-CG and one full Jacobi-CG solve to 1e-6, test "
                                      "microstructure 1000, load e1"},
            "note": "the oracle is a plain correctness reference (element loops, recursive DFT), not a tuned "
                    "CPU solver"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--train-seeds", type=int, default=64)
    ap.add_argument("--M", type=int, default=0, help="mode parameter (0 = pick from a small sweep)")
    ap.add_argument("--jac-steps", type=int, default=4)
    ap.add_argument("--no-oracle-ref", action="store_true", help="skip the FP64 oracle reference of kappa_bar")
    ap.add_argument("--no-autotune", action="store_true", help="operator shapes by rule instead of the autotuner")
    ap.add_argument("--march-shape", default="",
                    help="TZ,RY,XB: pin the FP64 operator march shape of the 48-load step (e.g. the autotuner's "
                         "pick of an earlier run) instead of tuning it; for counter runs, where the tuner's timings "
                         "are distorted")
    ap.add_argument("--no-calls", action="store_true", help="skip the standalone fe_apply / uno_precond_apply rooflines")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="most host cores the oracle's all-core baseline uses (one solve per core)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-192", action="store_true", help="skip the per-kernel roofline at 192^3")
    ap.add_argument("--no-elastic", action="store_true", help="skip the 128^3 elasticity record")
    ap.add_argument("--no-many", action="store_true", help="skip the many-problem record")
    ap.add_argument("--no-paper192", action="store_true", help="skip the 192^3 R = 5 record (the paper's size)")
    ap.add_argument("--only", choices=["elastic", "many", "paper192"], default=None,
                    help="run only that record and print it (profiling runs of its kernels)")
    ap.add_argument("--el-M", type=int, default=8, help="mode parameter of the elastic UNO preconditioner")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (reference for HBM counters)")
    return ap.parse_args()


def copy_rate(torch, dev, mib=2048, reps=5):
    """Achievable HBM rate on this device: a plain 2 GiB device-to-device copy
    (read + write bytes) timed with events, best of a few."""
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return round(2.0 * (mib << 20) / (best * 1e-3) / 1e9, 1)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every solve runs on a single MI355X "
              "(sharding over several GPUs is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2508_02681_amd as uno
    import synth_inputs as si

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    uno.lib()
    if args.calib_copy_mib > 0:  # a plain copy of known size: the scale of the FETCH/WRITE counters
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        recs = {"elastic": lambda: elastic_record(uno, si, torch, dev, args.el_M),
                "many": lambda: many_record(uno, si, torch, dev),
                "paper192": lambda: paper192_record(uno, si, torch, dev, not args.no_autotune)}
        rec = recs[args.only]()
        print(json.dumps({args.only: rec}), flush=True)
        return
    cfg = dict(si.CONFIG_3D_64)
    n_dof = int(np.prod(SHAPE))

    # ---------------- inputs (untimed) ----------------
    t0 = time.time()
    test_seeds = cfg["test_seeds"]
    kap_test = [torch.tensor(si.microstructure(cfg, s)[0], device=dev) for s in test_seeds]
    train_seeds = cfg["train_seeds"][: args.train_seeds]
    kap_train = [torch.tensor(si.microstructure(cfg, s)[0], device=dev) for s in train_seeds]
    log("inputs: %d test + %d train microstructures in %.1fs" % (len(kap_test), len(kap_train), time.time() - t0))

    # ---------------- training (untimed) ----------------
    t0 = time.time()
    hs = uno.half_shape(SHAPE)

    def solve_pairs(kaps, precond, kind):
        F, U, its = [], [], []
        for k in kaps:
            u, infos = uno.pcg_solve_batch(k, macro_loads=LOADS, kind=kind, precond=precond, rtol=1e-10,
                                           max_iter=20000)
            for j, g in enumerate(LOADS):
                F.append(uno.uno_macro_rhs(k, g))
                U.append(u[j])
                its.append(infos[j]["iters"])
        return F, U, its

    def fit(F, U, M):
        A = torch.zeros(hs, dtype=torch.float64, device=dev)
        B = torch.zeros(hs, dtype=torch.float64, device=dev)
        uno.uno_train_accumulate(torch.stack(F), torch.stack(U), A, B, len(F))
        return uno.uno_train_fit(SHAPE, M, A, B)

    # seeded random start: theta0^2 near the inverse Jacobi scale of the matrix phase
    M0 = 8
    h = 1.0 / SHAPE[0]
    scale = math.sqrt(1.0 / (8.0 * h / 3.0 * 8.0 * cfg["k_matrix"]))
    theta0 = si.random_theta(uno.num_weights(3, M0), 12345, scale=scale, spread=0.1)
    p0 = uno.UnoPrecond.create(SHAPE, M0, theta0)
    nboot = max(1, len(kap_train) // 4)
    F, U, its0 = solve_pairs(kap_train[:nboot], p0, "uno")
    theta1 = fit(F, U, M0)
    p1 = uno.UnoPrecond.create(SHAPE, M0, theta1)
    F2, U2, its1 = solve_pairs(kap_train[nboot:], p1, "uno")
    F += F2
    U += U2
    log("training pairs: %d (random-theta UNO-CG mean %.0f passes, refit UNO-CG mean %.0f)" %
        (len(F), np.mean(its0), np.mean(its1) if its1 else float("nan")))
    # mode parameter M (tuned, as in the paper): fastest time to tolerance on
    # held-out validation microstructures, solved as the benchmark's step
    # solves (every microstructure x every load in one batch)
    nval = len(test_seeds)
    kap_val = torch.stack([torch.tensor(si.microstructure(cfg, 5000 + i)[0], device=dev)
                           for i in range(nval) for _ in LOADS])
    loads_val = np.tile(LOADS, (nval, 1))
    Ms = [args.M] if args.M > 0 else [8, 12, 16, 20, 24]
    best = None
    for M in Ms:
        th = fit(F, U, M)
        p = uno.UnoPrecond.create(SHAPE, M, th)
        for rep in range(2):  # first pass warms up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, infos = uno.pcg_solve_batch(kap_val, macro_loads=loads_val, kind="uno", precond=p, rtol=RTOL,
                                           kappa_per_rhs=True)
            it = sum(i["iters"] for i in infos)
            torch.cuda.synchronize()
            tv = time.perf_counter() - t1
        log("  M=%d: %d passes, %.2f ms on validation (%d solves)" % (M, it, tv * 1e3, len(infos)))
        if best is None or tv < best[0]:
            best = (tv, M, th, p)
    _, M, theta, prec = best
    train_s = time.time() - t0
    log("trained M=%d in %.1fs" % (M, train_s))

    # one step = every test microstructure x every load: nm x 3 solves
    nm = len(kap_test)
    kap_all = torch.stack([k for k in kap_test for _ in LOADS])
    loads_all = np.tile(LOADS, (nm, 1))
    sols = torch.zeros((nm * len(LOADS),) + SHAPE, dtype=torch.float64, device=dev)
    nr_all = nm * len(LOADS)
    kap16 = torch.stack(kap_test)  # one field per microstructure, for the effective tensors
    worst_true = {}  # largest true relative residual ||f - A u|| / ||f|| (FP64) at exit, per solver

    def step(kind, precond, mode="all", tag="uno_cg", **kw):
        """The whole hot path over the test set: rhs + CG for every load of
        every microstructure, then kappa_bar of each.  mode "all": the nm x 3
        solves carried together by every pass kernel; "micro": the 3 loads of
        one microstructure together, microstructure after microstructure;
        "single": one load at a time."""
        sols.zero_()
        if mode == "all":
            _, infos = uno.pcg_solve_batch(kap_all, macro_loads=loads_all, u=sols, kind=kind, precond=precond,
                                           rtol=RTOL, max_iter=50000, kappa_per_rhs=True, **kw)
        elif mode == "micro":
            infos = []
            for i, k in enumerate(kap_test):
                infos += uno.pcg_solve_batch(k, macro_loads=LOADS, u=sols[3 * i: 3 * i + 3], kind=kind,
                                             precond=precond, rtol=RTOL, max_iter=50000, **kw)[1]
        else:
            infos = [uno.pcg_solve(kap_all[j], macro_load=loads_all[j], u=sols[j], kind=kind, precond=precond,
                                   rtol=RTOL, max_iter=50000, **kw)[1] for j in range(nr_all)]
        for info in infos:
            if not info["converged"]:
                raise RuntimeError("solve did not converge: %s" % info)
        worst_true[tag] = max(worst_true.get(tag, 0.0), max(info["true_rel_res"] for info in infos))
        kbs = list(uno.effective_tensor_batch(kap16, LOADS, sols))
        return [info["iters"] for info in infos], kbs

    def timed(kind, precond, steps, warmup, mode="all", tag="uno_cg", **kw):
        for _ in range(warmup):
            step(kind, precond, mode, tag, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        all_its, kbs = [], []
        for _ in range(steps):
            its, kb = step(kind, precond, mode, tag, **kw)
            all_its += its
            kbs += kb
        torch.cuda.synchronize()
        return time.perf_counter() - t, all_its, kbs

    # ---------------- operator shapes: the project's autotuner ----------------
    tuned = {}
    if args.march_shape:
        tz, ry, xb = (int(v) for v in args.march_shape.split(","))
        uno.set_operator_shape(SHAPE, nr_all, tz, ry, xb, kappa_per_rhs=True, dtype=torch.float64)
        tuned["f64"] = dict(tz=tz, ry=ry, xb=xb, pinned=True)
    if not args.no_autotune:
        for tag, dtp in (("f64", torch.float64), ("f32", torch.float32)):
            if tag not in tuned:
                tuned[tag] = uno.autotune_operator(SHAPE, nr_all, kappa_per_rhs=True, dtype=dtp)
        log("autotuned operator march (64^3 x %d): %s" % (nr_all, tuned))

    # ---------------- timed: UNO-CG FP64 (headline) ----------------
    dt, its, kbs = timed("uno", prec, args.steps, args.warmup)
    ms_step = dt / args.steps * 1e3
    value = n_dof * sum(its) / dt
    uno_t_solve = dt / len(its) * 1e3
    log("UNO-CG: %.2f ms/step (%d solves), %.1f passes/solve, %.3e DOF*it/s, %.3f ms per solve" %
        (ms_step, nr_all, np.mean(its), value, uno_t_solve))
    # the same solves three loads at a time, and one load at a time (context)
    dtq, itsq, _ = timed("uno", prec, 1, 1, mode="micro")
    micro_t_solve = dtq / len(itsq) * 1e3
    dts, itss, _ = timed("uno", prec, 1, 1, mode="single")
    seq_t_solve = dts / len(itss) * 1e3
    dtsg, itssg, _ = timed("uno", prec, 1, 1, mode="single", use_graphs=True)
    seq_t_solve_g = dtsg / len(itssg) * 1e3
    dtg, itsg, _ = timed("uno", prec, max(1, args.steps // 2), 1, use_graphs=True)
    all_t_solve_g = dtg / len(itsg) * 1e3
    log("UNO-CG 3 loads per launch: %.3f ms per solve; one load at a time: %.3f ms per solve (graphs %.3f); "
        "all %d together from graphs %.3f ms per solve" %
        (micro_t_solve, seq_t_solve, seq_t_solve_g, nr_all, all_t_solve_g))
    # ---------------- Jacobi-CG on the same microstructures ----------------
    dtj, itsj, kbj = timed("jacobi", None, args.jac_steps, 1, tag="jac_cg")
    jac_t_solve = dtj / len(itsj) * 1e3
    jac_rate = n_dof * sum(itsj) / dtj
    log("Jac-CG: %.1f passes/solve, %.3e DOF*it/s, %.3f ms per solve" % (np.mean(itsj), jac_rate, jac_t_solve))

    # ---------------- mixed precision: FP32 operator / preconditioner ----------------
    f32 = dict(op_dtype=torch.float32, prec_dtype=torch.float32)
    dtm, itsm, kbm = timed("uno", prec, 2, 1, tag="uno_cg_fp32", **f32)
    kb_err = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(kbm, kbs[:nm]))
    log("UNO-CG FP32 op/prec: %.1f passes/solve, %.3f ms per solve, kappa_bar rel diff vs FP64 %.1e" %
        (np.mean(itsm), dtm / len(itsm) * 1e3, kb_err))
    # where the FP32 step's time goes: every kernel family's summed launch
    # time over one step (the restarts' FP64 operator applies and transforms
    # are families of their own)
    f32_fams = {uno.KT_MATVEC: "operator march (FP32, CG)", uno.KT_UPDATE: "pass A + update (FP32 d, p)",
                uno.KT_FFT_MID: "pass B", uno.KT_FFT_INV: "pass C (FP32 s)",
                uno.KT_APPLY: "FP64 operator applies (residual replacement, exit check)",
                uno.KT_FFT_FWD: "pass A without update (restarts)"}
    ft32, _ = family_times(uno, f32_fams, lambda: step("uno", prec, "all", "uno_cg_fp32", **f32)[0])
    fp32_families = {name: {"ms_per_step": round(ft32[f][0], 3), "launches": int(ft32[f][1]),
                            "us_per_launch": round(ft32[f][0] / max(ft32[f][1], 1) * 1e3, 2)}
                     for f, name in f32_fams.items()}
    log("FP32 step by family (ms): %s of %.2f ms" % ({k: v["ms_per_step"] for k, v in fp32_families.items()},
                                                    dtm / 2 * 1e3))
    # the BF16 preconditioner mode: the FP32 mode with the learned-mode
    # passes' table and spectrum stored in BF16 (kept as the default only if
    # it costs no extra passes)
    bf16 = dict(op_dtype=torch.float32, prec_dtype=torch.bfloat16)
    dtb, itsb, kbb = timed("uno", prec, 2, 1, tag="uno_cg_bf16", **bf16)
    kb_err_b = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(kbb, kbs[:nm]))
    log("UNO-CG BF16 precond (FP32 op): %.1f passes/solve (FP32 mode %.1f), %.3f ms per solve, kappa_bar rel diff "
        "vs FP64 %.1e" % (np.mean(itsb), np.mean(itsm), dtb / len(itsb) * 1e3, kb_err_b))

    # ---------------- FANS (reference-medium preconditioner) for context ----------------
    pf = uno.UnoPrecond.fans(SHAPE, 0.5 * (cfg["k_matrix"] + cfg["k_incl"]))
    dtf, itsf, _ = timed("uno", pf, 1, 1, tag="fans_cg")
    log("FANS-CG: %.1f passes/solve, %.3f ms per solve" % (np.mean(itsf), dtf / len(itsf) * 1e3))

    # ---------------- dominant kernel: live HIP-event timing ----------------
    try:  # the learned-mode passes are in use when the table has them (AUTO == LEARNED then)
        prec.set_path(prec.PATH_LEARNED)
        learned = True
    except RuntimeError:
        learned = False
    prec.set_path(prec.PATH_AUTO)
    fams, bytes_per = kernel_families(uno, SHAPE, M, learned, True)
    roofline = roofline_record(fams, bytes_per, family_times(uno, fams, lambda: step("uno", prec)[0]))
    roofline["copy_GBs"] = copy_rate(torch, dev)
    if learned and kernel_sources_hash() == TRAFFIC_SRC:
        roofline["traffic"] = TRAFFIC_BYTES.get(roofline["kernel"])
    log("roofline (64^3): %s %.1f GB/s per launch (%.3f of peak)" %
        (roofline["kernel"], roofline["achieved"], roofline["frac"]))

    # ---------------- differentiation: d kappa_bar / d kappa_e, training step ----------------
    k0 = kap_test[0]
    ug, _ = uno.pcg_solve_batch(k0, macro_loads=LOADS, kind="uno", precond=prec, rtol=RTOL)
    jac = torch.empty((3, 3) + SHAPE, dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    uno.effective_tensor_grad(SHAPE, LOADS, ug, out=jac)
    ev0.record()
    for _ in range(10):
        uno.effective_tensor_grad(SHAPE, LOADS, ug, out=jac)
    ev1.record()
    torch.cuda.synchronize()
    g_ms = ev0.elapsed_time(ev1) / 10
    g_bytes = n_dof * 8 * (3 + 9)  # read the three solutions, write the 3 x 3 derivatives per voxel
    euler = torch.einsum("ijxyz,xyz->ij", jac, k0).cpu().numpy()
    kb0 = uno.effective_tensor(k0, LOADS, ug)
    grad_rec = {"workload": "d kappa_bar / d kappa_e, all %d voxels, 64^3 test microstructure 1000" % n_dof,
                "ms": round(g_ms, 4), "achieved_GBs": round(g_bytes / (g_ms * 1e-3) / 1e9, 1),
                "euler_identity_rel_err": float(np.abs(euler - kb0).max() / np.abs(kb0).max())}
    A = torch.zeros(hs, dtype=torch.float64, device=dev)
    B = torch.zeros_like(A)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    uno.uno_train_accumulate(torch.stack(F[:16]), torch.stack(U[:16]), A, B, 16)
    loss, gtheta = uno.uno_train_loss_grad(SHAPE, M, A, B, theta)
    torch.cuda.synchronize()
    grad_rec["training_step_batch16_ms"] = round((time.perf_counter() - t1) * 1e3, 3)
    log("d kappa_bar/d kappa: %.3f ms (%.0f GB/s), Euler identity %.1e; training step (16 pairs) %.2f ms" %
        (g_ms, grad_rec["achieved_GBs"], grad_rec["euler_identity_rel_err"], grad_rec["training_step_batch16_ms"]))

    # ---------------- 3D linear elasticity, 128^3 (c = 3) ----------------
    el = None
    if not args.no_elastic:
        el = elastic_record(uno, si, torch, dev, args.el_M)

    # ---------------- many problems of uneven sizes in one call ----------------
    many = None
    if not args.no_many:
        many = many_record(uno, si, torch, dev)

    # ---------------- the paper's size and contrast: 192^3, R = 5 ----------------
    paper192 = None
    if not args.no_paper192:
        paper192 = paper192_record(uno, si, torch, dev, not args.no_autotune)

    # ---------------- per-kernel roofline at the paper's grid size (192^3) ----------------
    big = None
    if not args.no_192:
        tuned192 = tune_192(uno, not args.no_autotune)
        cfgb = dict(cfg, shape=(192, 192, 192), r_min=12.0, r_max=24.0)
        kb192 = torch.tensor(si.microstructure(cfgb, 7000)[0], device=dev)
        pb = uno.UnoPrecond.create(cfgb["shape"], 12, si.random_theta(uno.num_weights(3, 12), 7001,
                                                                        scale=0.02, spread=0.1))
        fb, bb = kernel_families(uno, cfgb["shape"], 12, True, False)
        ub = torch.zeros((3,) + cfgb["shape"], dtype=torch.float64, device=dev)

        def run_big():
            ub.zero_()
            _, inf = uno.pcg_solve_batch(kb192, macro_loads=LOADS, u=ub, kind="uno", precond=pb, rtol=1e-30,
                                         max_iter=40)
            return [i["iters"] for i in inf]

        run_big()
        big = roofline_record(fb, bb, family_times(uno, fb, run_big))
        big["workload"] = "192^3, spheres r 12-24 vf 0.25, kappa 1/100, M = 12, three loads per launch, 40 passes"
        big["operator_shape_autotuned"] = tuned192.get(3)
        log("roofline (192^3): " + ", ".join("%s %.0f GB/s" % (k, v) for k, v in big["per_family_GBs"].items()))

    # ---------------- kappa_bar of every solver against the FP64 oracle ----------------
    oracle_err = None
    if not args.no_oracle_ref:
        oracle_err = oracle_kbar_errors(kap_test[0].cpu().numpy(),
                                        {"uno_cg": kbs[0], "jac_cg": kbj[0], "uno_cg_fp32": kbm[0],
                                         "uno_cg_bf16": kbb[0]})

    # ---------------- the C-ABI calls fe_apply and uno_precond_apply at 192^3 ----------------
    calls = None
    if not args.no_calls:
        calls = call_rooflines(uno, si, torch, dev, cfg)

    # ---------------- CPU baseline: the oracle, bounded sample ----------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_record([k.cpu().numpy() for k in kap_test], theta, M, n_dof, args.cpu_workers)

    out = {
        "metric": "DOF*iters/s (UNO-CG FP64, 3D 64^3, contrast 100, rel. residual 1e-6)",
        "value": value,
        "unit": "DOF*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D thermal 64^3 periodic hex8, spheres r 4-8 vf 0.25, kappa 1/100, "
                               "16 microstructures x 3 loads per step, solved together, UNO-CG to 1e-6 + effective tensors",
                   "grid": list(SHAPE), "loads_per_microstructure": 3, "solves_per_step": nr_all, "M": M,
                   "train_pairs": len(F), "operator_shape_autotuned": tuned,
                   "microstructures": len(kap_test)},
        "uno_cg": {"passes_mean": float(np.mean(its)), "ms_per_solve": uno_t_solve, "dof_iters_per_s": value,
                   "solves_per_launch": nr_all, "ms_per_solve_3_loads_per_launch": micro_t_solve,
                   "ms_per_solve_one_at_a_time": seq_t_solve,
                   "ms_per_solve_one_at_a_time_graphs": seq_t_solve_g,
                   "ms_per_solve_all_together_graphs": all_t_solve_g},
        "jac_cg": {"passes_mean": float(np.mean(itsj)), "ms_per_solve": jac_t_solve, "dof_iters_per_s": jac_rate},
        "fans_cg": {"passes_mean": float(np.mean(itsf)), "ms_per_solve": dtf / len(itsf) * 1e3},
        "uno_cg_fp32": {"passes_mean": float(np.mean(itsm)), "ms_per_solve": dtm / len(itsm) * 1e3,
                        "ms_per_step": dtm / 2 * 1e3, "kernel_families_one_step": fp32_families,
                        "kappa_bar_rel_diff_vs_fp64": kb_err},
        "uno_cg_bf16": {"passes_mean": float(np.mean(itsb)), "ms_per_solve": dtb / len(itsb) * 1e3,
                        "kappa_bar_rel_diff_vs_fp64": kb_err_b,
                        "note": "FP32 mode with the learned-mode passes' table, row-chunk partials and per-mode "
                                "coefficients stored in BF16 (FP64 arithmetic and recurrences)"},
        "kappa_bar_error_vs_fp64_oracle": oracle_err,
        "roofline_calls": calls,
        "time_to_tol_speedup_uno_vs_jac": jac_t_solve / uno_t_solve,
        "kappa_bar_first": np.round(kbs[0], 6).tolist(),
        "true_rel_res_max": worst_true,
        "roofline": roofline,
        "roofline_192": big,
        "differentiation": grad_rec,
        "elasticity_128": el,
        "many_problems": many,
        "paper_size_192_r5": paper192,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
