"""The seeded input generator: determinism, target volume fraction, and the
two-phase field (no GPU)."""
import numpy as np

import synth_inputs as si


def test_rsa_deterministic_and_fraction():
    a, fa = si.rsa_inclusions((32, 32), 3, 5, 0.3, 4)
    b, fb = si.rsa_inclusions((32, 32), 3, 5, 0.3, 4)
    assert np.array_equal(a, b) and fa == fb
    assert 0.3 <= fa < 0.45
    assert abs(a.mean() - fa) < 1e-12


def test_rsa_3d_config_shape():
    cfg = dict(si.CONFIG_3D_64)
    cfg["shape"] = (24, 24, 24)
    kap, frac = si.microstructure(cfg, 1000)
    assert kap.shape == (24, 24, 24)
    assert set(np.unique(kap)) <= {1.0, 100.0}
    assert frac >= 0.25


def test_laminate_layers():
    k = si.laminate((6, 4), 0, [1.0, 10.0])
    assert np.array_equal(k[:, 0], [1, 10, 1, 10, 1, 10])
    assert np.all(k == k[:, :1])
