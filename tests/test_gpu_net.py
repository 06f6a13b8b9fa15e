"""GPU tests of the warm-start network: its BF16 matrix-core forward and backward
kernels against the FP64 network oracle, the Adam step, training, and the warm
start modes of the inversion.

Tolerances.  The oracle with bf16=True rounds every convolution's operands to
bfloat16 as the matrix cores consume them and then works in FP64, so the forward
pass differs only by FP32 accumulation and by activations that fall on the other
side of a bfloat16 rounding boundary: relative L2 error below 5e-3.  The GPU
backward pass also feeds bfloat16 gradients to the matrix cores (the oracle's
backward keeps them in FP64, taking the rounding's derivative as one), a relative
perturbation of 2^-9 per operand that averages out over the sums: gradient
relative L2 error below 5e-3 overall and 1e-2 per layer, cosine above 0.9999.

Element by element (so that an error confined to a few sites, a tile edge or one
channel cannot hide under a norm): per output channel, max |difference| <= 1e-2 of the
channel's largest oracle value for the forward pass, and per layer max |difference| <=
1e-2 of the layer's largest oracle gradient (measured: at most 3.8e-3 and 2.3e-3).  A bfloat16 rounding that falls the other
way moves one operand by 2^-8 of itself; a handful of those in one 27 ci-term sum stays
well inside that, while a wrong halo, tile or channel offset moves values by O(1).
"""
import sys

import numpy as np
import pytest

from paper_1204_2088_amd import workloads as W

pytestmark = pytest.mark.gpu

WIDTHS = (8, 16, 24, 32)


@pytest.fixture(scope="module")
def hsf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1204_2088_amd import hsf as H
    H.load()
    return H


@pytest.fixture(scope="module")
def NO():
    from oracle import net_oracle
    return net_oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def smooth_inputs(B, C, L, seed, mean=0.5, amp=0.3):
    """Smooth random inputs [B][C][L][L][L] (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((B, C, L, L, L))
    for ax in (2, 3, 4):   # two passes of a periodic 3-point average per axis
        for _ in range(2):
            x = (np.roll(x, 1, ax) + x + np.roll(x, -1, ax)) / 3.0
    x /= np.std(x)
    return (mean + amp * x).astype(np.float32)


def oracle_out(NO, params, x, in_ch, out_ch, widths, bf16, shift=None, scale=None):
    import torch
    with torch.no_grad():
        y = NO.forward(params.astype(np.float64), torch.as_tensor(x.astype(np.float64)), in_ch, out_ch, widths,
                       bf16=bf16, shift=shift, scale=scale)
    return y.numpy()


@pytest.mark.parametrize("in_ch,out_ch,widths,B,L", [
    (3, 2, WIDTHS, 2, 16),
    (2, 3, (5, 12, 20, 32), 1, 24),     # ragged tiles on every level, odd widths
    (2, 2, (8, 8, 16, 16), 3, 8),       # 1^3 box on the coarsest level
    (4, 2, (8, 16), 2, 20),             # two levels, ragged 20^3 / 10^3 boxes
    (4, 2, (8, 16, 24), 1, 12),         # three levels down to 3^3
    (4, 2, (16,), 2, 9),                # one level (no pooling), odd box
])
def test_forward_matches_oracle(hsf, NO, in_ch, out_ch, widths, B, L):
    say(f"[net forward] in {in_ch} out {out_ch} widths {widths} B {B} L {L}")
    net = hsf.Net(in_ch, out_ch, widths, seed=11)
    p = net.get_params()
    # non-zero biases so their path is exercised too
    rng = np.random.Generator(np.random.PCG64(5))
    p = (p + 0.05 * rng.standard_normal(p.size)).astype(np.float32)
    net.set_params(p)
    shift = [0.5 - 0.1 * c for c in range(in_ch)]
    scale = [2.0 + c for c in range(in_ch)]
    net.set_input_norm(shift, scale)
    x = smooth_inputs(B, in_ch, L, seed=7)
    got = net.forward(x.ravel(), B, L).reshape(B, out_ch, L, L, L)
    ref = oracle_out(NO, p, x, in_ch, out_ch, widths, True, shift, scale)
    ref64 = oracle_out(NO, p, x, in_ch, out_ch, widths, False, shift, scale)
    e, e64 = rel_l2(got, ref), rel_l2(got, ref64)
    say(f"  rel L2 vs bf16 oracle {e:.3e}, vs fp64 oracle {e64:.3e}")
    assert np.all(np.isfinite(got))
    assert e < 5e-3
    assert e64 < 3e-2
    for c in range(out_ch):
        ec = float(np.max(np.abs(got[:, c] - ref[:, c])) / np.max(np.abs(ref[:, c])))
        say(f"  channel {c}: max |d| / max |ref| {ec:.3e}")
        assert ec <= 1e-2, c
    net.close()


@pytest.mark.parametrize("widths,L", [((16,), 32), ((8, 16, 24, 32), 16)])
def test_forward_from_device_and_host_agree(hsf, widths, L):
    """The forward pass reads device inputs in place (16-byte aligned ones with vector
    loads, others after a copy) and writes device outputs in place: every route gives
    the same bits as the host route, and the input buffer is left unchanged."""
    import torch
    say(f"[net forward routes] widths {widths} L {L}")
    B, in_ch, out_ch = 2, 4, 2
    net = hsf.Net(in_ch, out_ch, widths, seed=21)
    net.set_input_norm([0.5, 0.4, 0.0, 0.1], [3.0, 2.0, 1.5, 1.0])
    net.set_output_scale([2.0, 0.5])
    x = smooth_inputs(B, in_ch, L, seed=8).ravel()
    ref = net.forward(x, B, L)
    n = x.size
    for off in (0, 1, 2):   # offsets of 0, 4 and 8 bytes from a 256-byte aligned buffer
        buf = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
        buf[off:off + n] = torch.from_numpy(x).cuda()
        before = buf.clone()
        y = torch.full((B * out_ch * L ** 3,), float("nan"), dtype=torch.float32, device="cuda")
        net.forward(buf[off:off + n], B, L, out=y)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), ref), f"offset {off}"
        assert torch.equal(buf, before)
    net.close()


@pytest.mark.parametrize("B,L,widths", [(2, 16, WIDTHS), (4, 16, WIDTHS), (1, 24, WIDTHS), (2, 12, (8, 16)),
                                         (1, 12, (8, 12, 16)), (2, 7, (8,))])
def test_gradient_matches_oracle(hsf, NO, B, L, widths):
    in_ch, out_ch = 2, 2
    say(f"[net gradient] widths {widths} B {B} L {L}")
    net = hsf.Net(in_ch, out_ch, widths, seed=3)
    p = net.get_params()
    rng = np.random.Generator(np.random.PCG64(9))
    p = (p + 0.02 * rng.standard_normal(p.size)).astype(np.float32)
    net.set_params(p)
    net.set_input_norm([0.5, 0.5], [4.0, 4.0])
    x = smooth_inputs(B, in_ch, L, seed=21)
    t = smooth_inputs(B, out_ch, L, seed=22, mean=0.0, amp=1.0)
    loss, g = net.loss_grad(x.ravel(), t.ravel(), B, L)
    lref, gref = NO.loss_and_grad(p, x, t, in_ch, out_ch, widths, bf16=True, shift=[0.5, 0.5], scale=[4.0, 4.0])
    gref = np.asarray(gref)
    say(f"  loss gpu {loss:.8e} oracle {lref:.8e}")
    assert abs(loss - lref) <= 1e-3 * lref
    e = rel_l2(g, gref)
    say(f"  gradient rel L2 {e:.3e}")
    assert e < 5e-3
    off = 0
    for l, (ci, co) in enumerate(NO.layer_shapes(in_ch, out_ch, widths)):
        n = co * ci * 27 + co
        a, b = g[off:off + n].astype(np.float64), gref[off:off + n]
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        el = rel_l2(a, b)
        emax = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        say(f"  layer {l:2d} ({ci:2d}->{co:2d}) rel L2 {el:.3e} cosine {cos:.6f} max |d| / max |ref| {emax:.3e}")
        assert cos > 0.9999 and el < 1e-2, l
        assert emax <= 1e-2, l
        off += n


def test_adam_first_step_and_determinism(hsf):
    in_ch, out_ch, B, L = 2, 2, 1, 16
    x = smooth_inputs(B, in_ch, L, seed=1)
    t = smooth_inputs(B, out_ch, L, seed=2, mean=0.0)
    nets = [hsf.Net(in_ch, out_ch, WIDTHS, seed=4) for _ in range(2)]
    p0 = nets[0].get_params()
    _, g = nets[0].loss_grad(x.ravel(), t.ravel(), B, L)
    _, g2 = nets[0].loss_grad(x.ravel(), t.ravel(), B, L)
    assert np.array_equal(g, g2)   # fixed reduction order: bitwise repeatable
    lr = 1e-3
    nets[0].train_step(x.ravel(), t.ravel(), B, L, lr)
    p1 = nets[0].get_params()
    # first Adam step: m_hat = g, v_hat = g^2
    g64 = g.astype(np.float64)
    expect = p0 - lr * g64 / (np.abs(g64) + 1e-8)
    # the FP32 parameters round the result: allow two units in their last place
    assert np.all(np.abs(p1 - expect) <= 2 * np.spacing(np.abs(p0).astype(np.float32)) + 1e-6 * lr)
    # identical runs give identical parameters
    for net in nets:
        net.set_params(p0)
        for _ in range(5):
            net.train_step(x.ravel(), t.ravel(), B, L, lr)
    assert np.array_equal(nets[0].get_params(), nets[1].get_params())


def seeded_params(NO, in_ch, out_ch, widths, seed):
    """Parameters drawn on the host: weights uniform on +-sqrt(3 / fan_in), a quarter
    of that for the output layer, biases small."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    shapes = NO.layer_shapes(in_ch, out_ch, widths)
    for l, (ci, co) in enumerate(shapes):
        a = np.sqrt(3.0 / (27 * ci)) * (0.25 if l == len(shapes) - 1 else 1.0)
        out.append(rng.uniform(-a, a, co * ci * 27))
        out.append(0.01 * rng.standard_normal(co))
    return np.concatenate(out).astype(np.float32)


def training_problem(B, L, seed):
    """A smooth nonlinear, slightly nonlocal map of a two-channel input."""
    x = smooth_inputs(B, 2, L, seed=seed)
    xc = x.clip(0.05, None)
    t = np.stack([np.log(xc[:, 0] / xc[:, 1]), x[:, 0] - np.roll(x[:, 1], 1, axis=3)], axis=1)
    t = t.clip(-3, 3).astype(np.float32)
    assert np.all(np.isfinite(t))
    return x, t


def test_training_steps_match_oracle(hsf, NO):
    """Ten Adam steps on the GPU against the same steps taken by the FP64 oracle
    (bf16 operands) from the same host-drawn parameters."""
    B, L, lr = 2, 16, 1e-3
    x, t = training_problem(B, L, seed=31)
    p0 = seeded_params(NO, 2, 2, WIDTHS, seed=77)
    net = hsf.Net(2, 2, WIDTHS, seed=0)
    net.set_params(p0)
    net.set_input_norm([0.5, 0.5], [3.0, 3.0])
    p = p0.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for it in range(1, 11):
        lg = net.train_step(x.ravel(), t.ravel(), B, L, lr)
        lo, g = NO.loss_and_grad(p, x, t, 2, 2, WIDTHS, bf16=True, shift=[0.5, 0.5], scale=[3.0, 3.0])
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - lr * (m / (1 - 0.9 ** it)) / (np.sqrt(v / (1 - 0.999 ** it)) + 1e-8)
        say(f"  Adam step {it}: loss gpu {lg:.6e} oracle {lo:.6e}")
        assert abs(lg - lo) <= 3e-3 * lo, it
    e = rel_l2(net.get_params() - p0, p - p0)
    say(f"  parameter change after 10 steps: rel L2 difference {e:.3e}")
    assert e < 5e-2


def test_training_reduces_loss(hsf):
    """200 Adam steps (lr 1e-3) on the GPU fit the map: the loss falls at least
    sevenfold (the FP64 oracle, from the library's own initialisation, falls
    about seventeenfold) and never spikes."""
    B, L = 4, 16
    x, t = training_problem(B, L, seed=31)
    net = hsf.Net(2, 2, WIDTHS, seed=8)
    net.set_input_norm([0.5, 0.5], [3.0, 3.0])
    first = net.loss_grad(x.ravel(), t.ravel(), B, L, with_grad=False)[0]
    losses = []
    for it in range(200):
        losses.append(net.train_step(x.ravel(), t.ravel(), B, L, 1e-3))
        if it % 20 == 0:
            say(f"  step {it}: loss {losses[-1]:.4e}")
    last = net.loss_grad(x.ravel(), t.ravel(), B, L, with_grad=False)[0]
    say(f"[net training] loss {first:.4e} -> {last:.4e} after 200 Adam steps")
    assert all(np.isfinite(losses))
    assert max(losses) <= 1.5 * first
    assert last < first / 7


@pytest.mark.parametrize("warm", ["NET", "NET_DELTA", "NET_EXTRAP", "EXTRAP"])
def test_warm_modes_reach_the_same_solution(hsf, warm):
    """Whatever the starting fields, the inversion converges to the same fields (the
    map from densities to zero-mean fields is one to one)."""
    wl = W.melt16_a4b4()
    say(f"[warm {warm}] melt16_a4b4, 6 steps")
    phi = W.initial_composition(wl)
    w0 = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
    ctxs = []
    for mode in ("CURRENT", warm):
        ctx = hsf.Context(wl)
        ctx.set_densities(phi.ravel())
        ctx.set_fields(w0.ravel())
        if mode.startswith("NET"):
            in_ch = 2 if mode == "NET" else 4
            net = hsf.Net(in_ch, 2, WIDTHS, seed=1)
            net.set_input_norm([0.5] * in_ch, [10.0] * in_ch)
            ctx.attach_net(net)
        ctx.set_warm(getattr(hsf, "WARM_" + mode))
        ctxs.append(ctx)
    for k in range(6):
        out = [c.step(1, tol=1e-10, max_iter=2000) for c in ctxs]
        for st, _ in out:
            assert st[0]["converged"], (k, st)
        fa, fb = (c.get_fields() for c in ctxs)
        da, db = (c.get_densities() for c in ctxs)
        say(f"  step {k}: iterations {out[0][0][0]['iterations']} vs {out[1][0][0]['iterations']}, "
            f"max |dw| {np.max(np.abs(fa - fb)):.2e}")
        assert np.max(np.abs(fa - fb)) < 1e-6
        assert np.max(np.abs(da - db)) < 1e-9


def test_warm_start_formulas(hsf):
    """The starting fields of each warm start, read back after an inversion stopped
    at zero iterations, against the formulas computed on the host from the fields of
    the previous inversions (the network's output from its own forward call)."""
    wl = W.melt16_a4b4()
    V = wl.V
    base = W.initial_composition(wl)
    phis = [base]
    for k in range(1, 5):   # a slowly drifting sequence of target densities
        eta = W.random_fields((1,) + wl.shape, seed=40 + k, amplitude=0.004 * k, smooth=2)[0]
        p = base.copy()
        p[0] += eta - eta.mean()
        p[1] = 1.0 - p[0]
        phis.append(p)
    net = hsf.Net(4, 2, WIDTHS, seed=2)
    net.set_input_norm([0.5, 0.5, 0.0, 0.0], [8.0, 8.0, 1.0, 1.0])
    net_abs = hsf.Net(2, 2, WIDTHS, seed=3)
    net_abs.set_input_norm([0.5, 0.5], [8.0, 8.0])
    for mode in ("EXTRAP", "NET", "NET_DELTA", "NET_EXTRAP"):
        ctx = hsf.Context(wl)
        ctx.attach_net(net_abs if mode == "NET" else net)
        ctx.set_densities(phis[0].ravel())
        ctx.set_fields(np.zeros(2 * V))
        ws = []
        for k in range(3):
            ctx.set_densities(phis[k].ravel())
            st, _ = ctx.invert(tol=1e-11, max_iter=2000)
            assert st[0]["converged"]
            ws.append(ctx.get_fields().reshape(2, V))
        ctx.set_densities(phis[3].ravel())
        ctx.invert(tol=1e-11, max_iter=0, warm=getattr(hsf, "WARM_" + mode), allow_noconv=True)
        got = ctx.get_fields().reshape(2, V)
        w1, w2 = ws[1], ws[2]
        p1, p2, p3 = (phis[k].reshape(2, V) for k in (1, 2, 3))
        if mode == "EXTRAP":
            expect = 2 * w2 - w1
        elif mode == "NET":
            expect = net_abs.forward(p3.astype(np.float32).ravel(), 1, 16).reshape(2, V).astype(np.float64)
        else:
            delta = p3 - p2 if mode == "NET_DELTA" else p3 - 2 * p2 + p1
            r = np.sqrt(np.mean(delta ** 2))
            x = np.concatenate([p2, delta / r]).astype(np.float32)
            pred = net.forward(x.ravel(), 1, 16).reshape(2, V).astype(np.float64)
            expect = w2 + r * pred + ((w2 - w1) if mode == "NET_EXTRAP" else 0.0)
        expect -= expect.mean(axis=1, keepdims=True)   # the inversion fixes the gauge first
        err = np.max(np.abs(got - expect)) / np.max(np.abs(expect - w2))
        say(f"[warm formula {mode}] max error relative to the change {err:.2e}")
        assert err < 1e-6
        ctx.close()


def test_net_warm_start_rejects_bad_boxes(hsf):
    wl = W.melt16_a4b4().with_(L=(16, 16, 12))
    ctx = hsf.Context(wl)
    phi = W.initial_composition(wl)
    ctx.set_densities(phi.ravel())
    ctx.set_fields(np.zeros_like(phi).ravel())
    ctx.attach_net(hsf.Net(2, 2, WIDTHS, seed=1))
    with pytest.raises(hsf.HsfError):
        ctx.invert(tol=1e-8, warm=hsf.WARM_NET)
    ctx.attach_net(None)
    with pytest.raises(hsf.HsfError):
        ctx.invert(tol=1e-8, warm=hsf.WARM_NET)


def test_batched_replicas_network_warm_start(hsf):
    """Two replicas with equal boxes share one network call; the starting fields of
    each equal those of a context holding that replica alone."""
    wls = [W.melt16_a4b4().with_(seed=s) for s in (0, 1)]
    V = wls[0].V
    net = hsf.Net(4, 2, (8, 16), seed=5)
    net.set_input_norm([0.5, 0.5, 0.0, 0.0], [8.0, 8.0, 1.0, 1.0])

    def run(ws):
        ctx = hsf.Context(ws)
        ctx.attach_net(net)
        phis = [W.initial_composition(w) for w in ws]
        ctx.set_fields(np.zeros(2 * V * len(ws)))
        for k in range(4):
            p = np.concatenate([(ph * (1 + 0.01 * k * (ph - 0.5))).ravel() for ph in phis])
            ctx.set_densities(p)
            if k < 3:
                st, _ = ctx.invert(tol=1e-10, max_iter=2000)
                assert all(s["converged"] for s in st)
            else:
                ctx.invert(tol=1e-10, max_iter=0, warm=hsf.WARM_NET_EXTRAP, allow_noconv=True)
        out = ctx.get_fields().reshape(len(ws), 2, V)
        ctx.close()
        return out

    both = run(wls)
    for r, w in enumerate(wls):
        alone = run([w])[0]
        err = np.max(np.abs(both[r] - alone)) / np.max(np.abs(alone))
        say(f"[batched warm start] replica {r}: max rel difference {err:.2e}")
        assert err < 1e-12


def test_output_scale(hsf):
    """The output scale multiplies each output channel after the last convolution, and
    training is refused while a scale other than 1 is set."""
    net = hsf.Net(2, 2, (8, 16), seed=3)
    x = smooth_inputs(1, 2, 16, seed=4)
    t = smooth_inputs(1, 2, 16, seed=5)
    y1 = net.forward(x.ravel(), 1, 16).reshape(2, -1)
    net.set_output_scale([3.0, 0.25])
    y2 = net.forward(x.ravel(), 1, 16).reshape(2, -1)
    assert np.array_equal(y2[0], y1[0] * np.float32(3.0)) and np.array_equal(y2[1], y1[1] * np.float32(0.25))
    with pytest.raises(hsf.HsfError):
        net.train_step(x.ravel(), t.ravel(), 1, 16, 1e-3)
    net.set_output_scale([1.0, 1.0])
    net.train_step(x.ravel(), t.ravel(), 1, 16, 1e-3)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_sample_assembly_matches_numpy(hsf, mode):
    """The training samples, channel statistics and target scaling the library assembles
    on the device against the header's formulas evaluated with numpy in FP64: mode 0,
    x = phi and y = the two polymer fields; modes 1 and 2, x = (phi_n, delta phi / r),
    y = delta w / r over the two polymer fields, delta the first (mode 1) or second
    (mode 2) difference and r the rms of delta phi over species and sites; the per-channel
    mean and rms over samples and sites; x_c = (x_c - shift_c) scale_c.  A ragged box of
    40 x 41 x 17 sites (several hundred blocks per launch); the FP32 outputs within 1e-6
    relative of the FP64 values (one rounding)."""
    import torch
    rng = np.random.default_rng(31 + mode)
    nsp, V = 3, 40 * 41 * 17
    st = [rng.uniform(0.0, 1.0, nsp * V) for _ in range(3)]
    ws = [rng.standard_normal(nsp * V) for _ in range(3)]
    dev = [torch.as_tensor(a, device="cuda") for a in st + ws]
    phi, phi_n, phi_p, w, w_n, w_p = dev
    cin = nsp if mode == 0 else 2 * nsp
    net = hsf.Net(cin, 2, (8,), seed=2)
    B = 3
    x = torch.empty(B, cin, V, dtype=torch.float32, device="cuda")
    y = torch.empty(B, 2, V, dtype=torch.float32, device="cuda")
    for b in range(B):   # shifted copies make distinct samples
        net.make_sample(phi, phi_n if mode >= 1 else None, phi_p if mode == 2 else None, torch.roll(w, b),
                        w_n if mode >= 1 else None, w_p if mode == 2 else None, nsp, V, mode, x[b], y[b])
    torch.cuda.synchronize()
    if mode == 0:
        r, xr = 1.0, st[0]
    else:
        dphi = st[0] - st[1] if mode == 1 else st[0] - 2 * st[1] + st[2]
        r = np.sqrt(np.mean(dphi ** 2))
        xr = np.concatenate([st[1], dphi / r])
    got = x.cpu().numpy().astype(np.float64)
    for b in range(B):
        wb = np.roll(ws[0], b)
        dw = wb if mode == 0 else ((wb - ws[1]) if mode == 1 else (wb - 2 * ws[1] + ws[2]))
        assert np.max(np.abs(got[b].ravel() - xr)) <= 1e-6 * np.max(np.abs(xr))
        yr = dw[:2 * V] / r
        assert np.max(np.abs(y[b].cpu().numpy().astype(np.float64).ravel() - yr)) <= 1e-6 * np.max(np.abs(yr))
    mean, rms = net.channel_moments(x, B, cin, V)
    for c in range(cin):
        v = got[:, c, :]
        assert abs(mean[c] - v.mean()) <= 1e-12 * (1 + abs(v.mean()))
        assert abs(rms[c] - np.sqrt(np.mean(v ** 2))) <= 1e-12 * np.sqrt(np.mean(v ** 2))
    shift = [0.25 * c for c in range(cin)]
    scale = [1.0 / (1.0 + c) for c in range(cin)]
    want = (x.cpu().numpy() - np.array(shift, np.float32)[None, :, None]) * np.array(scale, np.float32)[None, :, None]
    net.affine(x, B, cin, V, shift, scale)
    torch.cuda.synchronize()
    d = np.abs(x.cpu().numpy().astype(np.float64) - want.astype(np.float64))
    assert np.max(d) <= 1e-6 * np.max(np.abs(want))
    say(f"[sample mode {mode}] r {r:.4f}; moments {np.round(mean, 4)} / {np.round(rms, 4)}")
