"""FP64 CPU reference of the warm-start network (plain PyTorch CPU operations).

TEST INFRASTRUCTURE ONLY (imported by the test suite).  It shares no code with the
HIP library: it builds the same topology from torch.nn.functional primitives on
float64 tensors and differentiates it with autograd.  With `bf16=True` the
operands of every convolution (input and weights) are rounded to bfloat16 before
the float64 convolution, which is what the GPU's matrix cores consume.

Topology (D = 1..4 levels, widths w1..wD; c(.) = SiLU(periodic 3x3x3 convolution + bias)):
  e1 = c(c(x)); el = c(c(pool e(l-1))) for l = 2..D
  dD = eD; dl = c(c(up d(l+1)) + el) for l = D-1..1; out = conv(d1)
pool: 2x2x2 average; up: nearest.  Parameter vector layout: per convolution (in the
order above, 4 D - 1 of them) W[co][ci][27] with k = 9 (dz+1) + 3 (dy+1) + (dx+1), then
b[co].  Widths are given as a sequence of D positive values (trailing zeros ignored).
"""
import numpy as np
import torch
import torch.nn.functional as F


def levels(widths):
    w = []
    for v in widths:
        if v <= 0:
            break
        w.append(int(v))
    return w


def layer_shapes(in_ch, out_ch, widths):
    w = levels(widths)
    D = len(w)
    shapes, prev = [], in_ch
    for l in range(D):
        shapes += [(prev, w[l]), (w[l], w[l])]
        prev = w[l]
    for l in range(D - 2, -1, -1):
        shapes += [(w[l + 1], w[l]), (w[l], w[l])]
    shapes.append((w[0], out_ch))
    return shapes


def num_params(in_ch, out_ch, widths):
    return sum(co * ci * 27 + co for ci, co in layer_shapes(in_ch, out_ch, widths))


def unpack(params, in_ch, out_ch, widths):
    """List of (W[co][ci][3][3][3], b[co]) float64 tensors from the flat vector."""
    p = params if isinstance(params, torch.Tensor) else torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, off = [], 0
    for ci, co in layer_shapes(in_ch, out_ch, widths):
        n = co * ci * 27
        W = p[off:off + n].reshape(co, ci, 3, 3, 3)   # [kz][ky][kx] = offsets (dz+1, dy+1, dx+1)
        off += n
        b = p[off:off + co]
        off += co
        out.append((W, b))
    return out


def to_bf16(t):
    """Value rounded to bfloat16 (round to nearest even); the derivative of the
    rounding is taken as one, so gradients pass through it unrounded in float64."""
    r = t.detach().to(torch.bfloat16).to(torch.float64)
    return t + (r - t.detach())


def conv_periodic(x, W, b, bf16=False):
    """out[o][x] = b[o] + sum_{c,k} W[o][c][k] x[c][x + off_k] on a periodic box
    (cross-correlation, as the forward convolution of the network)."""
    if bf16:
        x, W = to_bf16(x), to_bf16(W)
    xp = F.pad(x, (1, 1, 1, 1, 1, 1), mode="circular")
    return F.conv3d(xp, W, b)


def forward(params, x, in_ch, out_ch, widths, bf16=False, shift=None, scale=None):
    """x: float64 tensor [B][in_ch][L][L][L] -> [B][out_ch][L][L][L].  The input is
    first normalised per channel, (x - shift) * scale (identity by default)."""
    layers = unpack(params, in_ch, out_ch, widths) if not isinstance(params, list) else params
    if shift is not None:
        x = (x - torch.as_tensor(shift, dtype=torch.float64).reshape(1, -1, 1, 1, 1)) * \
            torch.as_tensor(scale, dtype=torch.float64).reshape(1, -1, 1, 1, 1)
    c = lambda i, h: F.silu(conv_periodic(h, *layers[i], bf16=bf16))
    pool = lambda h: F.avg_pool3d(h, 2)
    up = lambda h: h.repeat_interleave(2, 2).repeat_interleave(2, 3).repeat_interleave(2, 4)
    D = len(levels(widths))
    enc, h = [], x
    for l in range(D):
        h = c(2 * l + 1, c(2 * l, h if l == 0 else pool(h)))
        enc.append(h)
    i = 2 * D
    for l in range(D - 2, -1, -1):
        h = c(i + 1, c(i, up(h)) + enc[l])
        i += 2
    return conv_periodic(h, *layers[i], bf16=bf16)


def loss_and_grad(params, x, target, in_ch, out_ch, widths, bf16=False, shift=None, scale=None):
    """Mean square error over all outputs and its gradient (flat, float64)."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    layers = unpack(p, in_ch, out_ch, widths)
    out = forward(layers, torch.as_tensor(x, dtype=torch.float64), in_ch, out_ch, widths, bf16, shift, scale)
    t = torch.as_tensor(target, dtype=torch.float64)
    loss = ((out - t) ** 2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.detach().numpy().copy()
