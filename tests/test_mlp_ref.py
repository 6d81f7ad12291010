"""Pins of the CPU FP64 reference perceptron used to check the GPU kernels."""
import numpy as np

import mlp_ref
from paper_1812_04719_amd import toi_model


def test_reference_gradient_vs_central_differences():
    rng = np.random.default_rng(3)
    p = toi_model.init_params(1).astype(np.float64)
    p += rng.normal(0, 0.05, p.shape)
    x = rng.normal(0, 1, (40, 18))
    s = rng.uniform(0, 1, 40)
    g = mlp_ref.grad(p, x, s)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp_ref.loss(p + e, x, s) - mlp_ref.loss(p - e, x, s)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_rounding_nearest_even():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0], dtype=np.float32)
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 0.0])
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1
    want[1] = 1.0
    want[2] = 1.0 + 2 ** -6
    assert np.array_equal(mlp_ref.bf16(v), want)
