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


@pytest.mark.parametrize("widths", [(3,), (3, 4), (2, 3, 4), (2, 3, 2, 3)])
def test_shift_equivariance_matches_depth(widths):
    """A periodic U-Net of D levels commutes with translations by multiples of
    2^(D-1) sites (pooling and upsampling are aligned to that grid) and, for D >= 2,
    not with a one-site translation: a misaligned pooling or upsampling index, or a
    dropped level, breaks one of the two."""
    rng = np.random.default_rng(3)
    D = len(widths)
    n = NO.num_params(2, 2, widths)
    p = 0.4 * rng.standard_normal(n)
    x = torch.tensor(rng.standard_normal((1, 2, 8, 8, 8)))
    y = NO.forward(p, x, 2, 2, widths)
    q = 2 ** (D - 1)
    for ax in (2, 3, 4):
        ys = NO.forward(p, torch.roll(x, q, ax), 2, 2, widths)
        assert float(torch.max(torch.abs(ys - torch.roll(y, q, ax)))) < 1e-12
    if D >= 2:
        y1 = NO.forward(p, torch.roll(x, 1, 4), 2, 2, widths)
        assert float(torch.max(torch.abs(y1 - torch.roll(y, 1, 4)))) > 1e-3


def test_depth_layer_counts():
    for D, widths in enumerate([(4,), (4, 6), (4, 6, 8), (4, 6, 8, 10)], start=1):
        shapes = NO.layer_shapes(3, 2, widths)
        assert len(shapes) == 4 * D - 1
        assert shapes[0] == (3, 4) and shapes[-1] == (4, 2)
        # every layer reads its predecessor's width (a decoder skip adds an encoder
        # activation of that same width)
        assert all(shapes[i][0] == shapes[i - 1][1] for i in range(1, len(shapes)))
    assert NO.layer_shapes(3, 2, (4, 6, 0, 0)) == NO.layer_shapes(3, 2, (4, 6))
