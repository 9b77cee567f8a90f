"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the method: it only draws microstructures,
random vectors and random weight vectors from seeds.  Both the tests of the
HIP path and the oracle take their inputs from here.

Microstructures stand in for the paper's voxel datasets (2D 400^2 and
3D 192^3 two-phase images, Sec. 5), which are not available: two-phase
periodic images made of non-overlapping random inclusions (circles in 2D,
spheres in 3D) placed by random sequential addition.

Recipe (``rsa_inclusions``):
  * centres uniform in [0, N)^d, radius uniform in [r_min, r_max] voxels;
  * an inclusion is accepted if its minimum-image centre distance to every
    accepted inclusion is at least the sum of the two radii (no overlap,
    periodic);
  * a voxel belongs to an inclusion if its centre (i + 1/2) lies within the
    radius under the minimum-image convention;
  * stop when the voxel fraction reaches the target, or after 100000
    attempts; the achieved fraction is returned.
"""
from __future__ import annotations

import numpy as np

MAX_ATTEMPTS = 100_000


def rsa_inclusions(shape, r_min, r_max, volume_fraction, seed):
    """Return (phase uint8 array, achieved volume fraction); 1 = inclusion."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    rng = np.random.default_rng(seed)
    phase = np.zeros(shape, dtype=np.uint8)
    N = np.array(shape, dtype=np.float64)
    centres, radii = [], []
    total = float(np.prod(shape))
    filled = 0
    for _ in range(MAX_ATTEMPTS):
        if filled / total >= volume_fraction:
            break
        c = rng.uniform(0.0, 1.0, size=d) * N
        r = rng.uniform(r_min, r_max)
        ok = True
        for c2, r2 in zip(centres, radii):
            delta = np.abs(c - c2)
            delta = np.minimum(delta, N - delta)
            if float(np.sqrt(np.sum(delta * delta))) < r + r2:
                ok = False
                break
        if not ok:
            continue
        centres.append(c)
        radii.append(r)
        # paint voxels whose centres lie within r (minimum image)
        ranges = []
        for b in range(d):
            lo = int(np.floor(c[b] - r - 1))
            hi = int(np.ceil(c[b] + r + 1))
            ranges.append(np.arange(lo, hi + 1))
        grids = np.meshgrid(*ranges, indexing="ij")
        dist2 = np.zeros(grids[0].shape)
        for b in range(d):
            dd = np.abs(grids[b] + 0.5 - c[b])
            dd = np.minimum(dd, N[b] - dd)
            dist2 += dd * dd
        inside = dist2 <= r * r
        idx = tuple(np.mod(grids[b][inside], shape[b]) for b in range(d))
        before = int(phase[idx].sum())
        phase[idx] = 1
        filled += int(phase[idx].sum()) - before
    return phase, filled / total


def two_phase_kappa(phase, k_matrix, k_inclusion):
    """Phase-wise constant conductivity field (Sec. 5.1)."""
    return np.where(phase > 0, float(k_inclusion), float(k_matrix)).astype(np.float64)


def laminate(shape, axis, values, seed=None):
    """Voxel-aligned layers normal to ``axis``; layer i has values[i % len]."""
    shape = tuple(int(s) for s in shape)
    k = np.empty(shape, dtype=np.float64)
    vals = np.asarray(values, dtype=np.float64)
    if seed is not None:
        rng = np.random.default_rng(seed)
        per_layer = vals[rng.integers(0, len(vals), size=shape[axis])]
    else:
        per_layer = vals[np.arange(shape[axis]) % len(vals)]
    sl = [None] * len(shape)
    sl[axis] = slice(None)
    k[...] = per_layer[tuple(sl)]
    return k


def random_field(shape, seed, low=None, high=None):
    rng = np.random.default_rng(seed)
    if low is None:
        return rng.standard_normal(size=tuple(shape))
    return rng.uniform(low, high, size=tuple(shape))


def random_theta(num, seed, scale=1.0, spread=0.5):
    """Seeded weight vector theta_i = scale (1 + spread xi_i), xi ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    return scale * (1.0 + spread * rng.standard_normal(size=int(num)))


# Workloads of the benchmark and of the parity tests (sizes, contrasts, seeds).
CONFIG_2D_32 = dict(shape=(32, 32), r_min=3.0, r_max=5.0, vf=0.3, k_matrix=1.0, k_incl=10.0,
                    seeds=list(range(8)), loads=2)
CONFIG_3D_64 = dict(shape=(64, 64, 64), r_min=4.0, r_max=8.0, vf=0.25, k_matrix=1.0, k_incl=100.0,
                    train_seeds=list(range(64)), test_seeds=list(range(1000, 1016)), loads=3)


# 3D linear elasticity: Young's modulus 1 in the matrix and 100 in the
# spheres, Poisson's ratio 0.3 in both phases, six unit Mandel strain loads
CONFIG_EL_128 = dict(shape=(128, 128, 128), r_min=8.0, r_max=16.0, vf=0.25, k_matrix=1.0, k_incl=100.0, nu=0.3,
                     train_seeds=[5001, 5002], test_seeds=[5000], loads=6)


# the paper's 3D thermal size and contrast (192^3, kappa 1 in the matrix and
# 0.2 in the inclusions, R = 5) with this generator's spheres: context next
# to the paper's published timings, not a parity case
CONFIG_3D_192_R5 = dict(shape=(192, 192, 192), r_min=12.0, r_max=24.0, vf=0.25, k_matrix=1.0, k_incl=0.2,
                        train_seeds=[8001, 8002, 8003, 8004], val_seed=8010, test_seed=8000, loads=3)


# many-query work list: grid sizes mixed over 2D and 3D, inclusion radii
# N/16..N/8 voxels, contrast log-uniform in [10, 1000], 2 loads in 2D and 3
# in 3D
CONFIG_MANY = dict(count=256, shapes=[(64, 64), (128, 128), (256, 256), (32, 32, 32), (48, 48, 48)], vf=0.25,
                   contrast=(10.0, 1000.0), seed=7000, train_per_shape=4)


def many_problem(cfg, i):
    """Problem i of the work list: (conductivity field, loads)."""
    rng = np.random.default_rng(cfg["seed"] + 7919 * i)
    shape = cfg["shapes"][int(rng.integers(len(cfg["shapes"])))]
    lo, hi = cfg["contrast"]
    contrast = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    n0 = shape[0]
    ph, _ = rsa_inclusions(shape, n0 / 16.0, n0 / 8.0, cfg["vf"], cfg["seed"] + i)
    return two_phase_kappa(ph, 1.0, contrast), np.eye(len(shape))


def microstructure(cfg, seed):
    phase, frac = rsa_inclusions(cfg["shape"], cfg["r_min"], cfg["r_max"], cfg["vf"], seed)
    return two_phase_kappa(phase, cfg["k_matrix"], cfg["k_incl"]), frac
