"""Pins of the network oracle (CPU): the periodic convolution against an explicit
sum, the gradient against central finite differences, and the parameter count."""
import itertools

import numpy as np
import pytest
import torch

from oracle import net_oracle as NO


def test_periodic_conv_is_explicit_sum():
    rng = np.random.default_rng(0)
    L, ci, co = 4, 2, 3
    x = rng.standard_normal((1, ci, L, L, L))
    W = rng.standard_normal((co, ci, 27))
    b = rng.standard_normal(co)
    got = NO.conv_periodic(torch.tensor(x), torch.tensor(W.reshape(co, ci, 3, 3, 3)), torch.tensor(b)).numpy()
    ref = np.zeros((1, co, L, L, L))
    for o, z, y, xx in itertools.product(range(co), range(L), range(L), range(L)):
        s = b[o]
        for c in range(ci):
            for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
                k = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                s += W[o, c, k] * x[0, c, (z + dz) % L, (y + dy) % L, (xx + dx) % L]
        ref[0, o, z, y, xx] = s
    assert np.max(np.abs(got - ref)) < 1e-12


def test_parameter_count():
    pairs = [(3, 8), (8, 8), (8, 16), (16, 16), (16, 24), (24, 24), (24, 32), (32, 32), (32, 24), (24, 24),
             (24, 16), (16, 16), (16, 8), (8, 8), (8, 2)]
    assert NO.num_params(3, 2, (8, 16, 24, 32)) == sum(27 * a * b + b for a, b in pairs) == 146490
    assert NO.num_params(2, 2, (2, 2, 2, 2)) == sum(co * ci * 27 + co for ci, co in NO.layer_shapes(2, 2, (2, 2, 2, 2)))


def test_gradient_finite_differences():
    rng = np.random.default_rng(1)
    widths = (2, 3, 2, 3)
    n = NO.num_params(2, 2, widths)
    p = 0.3 * rng.standard_normal(n)
    x = rng.standard_normal((1, 2, 8, 8, 8))
    t = rng.standard_normal((1, 2, 8, 8, 8))
    loss, g = NO.loss_and_grad(p, x, t, 2, 2, widths)
    h = 1e-6
    for i in rng.choice(n, size=12, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = NO.loss_and_grad(pp, x, t, 2, 2, widths)
        lm, _ = NO.loss_and_grad(pm, x, t, 2, 2, widths)
        assert abs((lp - lm) / (2 * h) - g[i]) < 1e-6 * max(1.0, abs(g[i]))


def test_bf16_rounding_is_small():
    rng = np.random.default_rng(2)
    widths = (4, 4, 4, 4)
    n = NO.num_params(3, 2, widths)
    p = 0.2 * rng.standard_normal(n)
    x = torch.tensor(rng.uniform(0, 1, (1, 3, 8, 8, 8)))
    a = NO.forward(p, x, 3, 2, widths)
    b = NO.forward(p, x, 3, 2, widths, bf16=True)
    rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(a))
    assert 0 < rel < 2e-2
