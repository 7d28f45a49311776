"""Seeded input generators: determinism, shapes and the stated recipes."""
import math

import numpy as np

from paper_1206_3215_amd import inputs


def test_grid_excludes_right_end():
    X, Y = inputs.grid(4, 2, inputs.Domain(8.0, 2.0, -4.0, -1.0))
    assert X.shape == (2, 4)
    assert list(X[0]) == [-4.0, -2.0, 0.0, 2.0] and list(Y[:, 0]) == [-1.0, 0.0]


def test_nls_and_sg_inputs_deterministic():
    d = inputs.PAPER_DOMAIN
    a = inputs.nls_gaussian(64, 32, d, seed=4)
    b = inputs.nls_gaussian(64, 32, d, seed=4)
    assert a.shape == (32, 64) and a.dtype == np.complex128 and np.array_equal(a, b)
    assert not np.array_equal(a, inputs.nls_gaussian(64, 32, d, seed=5))
    u, v = inputs.sg_gaussian(32, 32, d, seed=0)
    assert u.dtype == np.float64 and not v.any()
    # noise-free peak is 0.5 at the origin (grid point j = n/2)
    assert inputs.nls_gaussian(32, 32, d, seed=None)[16, 16] == 0.5


def test_taylor_green_values():
    w = inputs.taylor_green(8, t=0.1, nu=0.1)
    assert abs(w[2, 2] - 4 * math.pi * math.exp(-8 * math.pi ** 2 * 0.01)) < 1e-14


def test_serving_mix_recipe():
    reqs = inputs.serving_mix(512, rate_hz=20.0)
    assert len(reqs) == 512
    assert {r.eq for r in reqs} == {"nls", "sg", "ns"}
    assert {r.n for r in reqs} <= {128, 256, 512, 1024, 2048}
    assert all(100 <= r.steps <= 2000 for r in reqs)
    arr = np.array([r.arrival_s for r in reqs])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    assert abs(len(reqs) / arr[-1] - 20.0) < 3.0
    assert reqs == inputs.serving_mix(512, rate_hz=20.0)
