"""Host logic of the benchmark (no GPU): the algorithmic bytes of the pass
kernels and the roofline record built from per-family event times, with
each load counted for the passes it ran."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


class KT:  # the kernel-family identifiers the binding exports
    KT_MATVEC, KT_UPDATE, KT_FFT_FWD, KT_FFT_MID, KT_FFT_INV = 1, 2, 3, 4, 5


def test_learned_flow_bytes_per_node():
    shape, M = (8, 6, 10), 2
    n = int(np.prod(shape))
    fams, bp = bench.kernel_families(KT, shape, M, True, True)
    assert set(fams) == {KT.KT_MATVEC, KT.KT_UPDATE, KT.KT_FFT_MID, KT.KT_FFT_INV}
    nblk = shape[0] * (2 * M + 1) * (M + 1)
    assert bp[KT.KT_MATVEC] == (40 * n, 0)               # s, d_old, kappa in; d_new, p out
    assert bp[KT.KT_UPDATE] == (48 * n + 16 * nblk, 0)   # r, u, d, p in; r, u out; block spectrum
    assert bp[KT.KT_FFT_INV] == (16 * n + 16 * nblk, 0)  # r, H in; s out
    # one conductivity field for all loads: read once per launch
    _, bp1 = bench.kernel_families(KT, shape, M, True, False)
    assert bp1[KT.KT_MATVEC] == (32 * n, 8 * n)


def test_roofline_counts_each_load_for_its_passes():
    shape, M = (8, 8, 8), 2
    fams, bp = bench.kernel_families(KT, shape, M, True, True)
    # two loads that ran 3 and 5 passes, 5 launches per family; the operator
    # takes the most time
    fam_ms = {f: (1.0, 5) for f in fams}
    fam_ms[KT.KT_MATVEC] = (2.0, 5)
    rec = bench.roofline_record(fams, bp, (fam_ms, [3, 5]))
    per_rhs, per_launch = bp[KT.KT_MATVEC]
    total = 8 * per_rhs + 5 * per_launch
    assert rec["kernel"] == fams[KT.KT_MATVEC]
    assert abs(rec["achieved"] - round(total / 2e-3 / 1e9, 1)) < 0.11
    assert rec["bytes_per_launch"] == round(total / 5)
    assert abs(rec["avg_us"] - 400.0) < 1e-9
    assert rec["peak"] == bench.HBM_PEAK_GBS and rec["bound"] == "hbm"
    assert abs(rec["frac"] - round(rec["achieved"] / bench.HBM_PEAK_GBS, 4)) < 1e-12
