"""Learned warm start of the inversion: training data from the inversion's own
converged results, training with the library's network kernels (hsf.Net), and the
comparison of the warm starts on a held-out trajectory.

The network predicts the linear response of the inversion: given the densities
phi^n of the latest inversion and a density difference delta (first difference
phi^(n+1) - phi^n, or second difference phi^(n+1) - 2 phi^n + phi^(n-1)) scaled to
unit rms r, it returns the matching field difference divided by r.  The library
applies it as HSF_WARM_NET_DELTA (w^n + r net) or HSF_WARM_NET_EXTRAP
(2 w^n - w^(n-1) + r net(second difference)), then runs the same inversion to the
same residual; the network only moves the starting point.

Everything here runs on the GPU through the library: the trajectories (hsf.Context), the
sample assembly, normalisation statistics and target scaling (hsf_net_make_sample,
hsf_net_channel_moments, hsf_net_affine) and the training (hsf.Net); torch only holds the
device memory.
"""
from __future__ import annotations

import time

import numpy as np

from . import hsf
from . import workloads as W

# One level of 16 channels: the inversion's linear response reaches a few lattice
# sites (about the chain's radius of gyration), which a single level covers; deeper
# networks were no more accurate on held-out trajectories and cost more per step.
DEFAULT_WIDTHS = (16,)


def _torch():
    import torch
    return torch


def initial_state(ctx, wls):
    """Field-layout arrays (densities, fields) of the workloads' initial compositions,
    with the local ideal-gas fields as the first guess."""
    phi = np.empty(ctx.nsp * ctx.T)
    w = np.empty(ctx.nsp * ctx.T)
    for r, wl in enumerate(wls):
        p = W.initial_composition(wl)
        fo = ctx.field_offset(r)
        n = ctx.nsp * wl.V
        phi[fo:fo + n] = p.ravel()
        w[fo:fo + n] = (-np.log(p / p.mean(axis=tuple(range(1, p.ndim)), keepdims=True))).ravel()
    return phi, w


def record_trajectory(wls, steps, record, tol=1e-10, precision="fp64", log=None, precond=False):
    """Run the coupled dynamics of the replicas `wls` for `steps` steps (extrapolated
    warm start) and keep, for every step index in `record`, the target densities and
    converged fields of that step's inversion as device tensors [rep][nsp][V] (FP64).
    Returns {k: (phi, w)}."""
    torch = _torch()
    ctx = hsf.Context(wls, precision=precision)
    ctx.set_solver(precond=precond)
    phi0, w0 = initial_state(ctx, wls)
    ctx.set_densities(phi0)
    ctx.set_fields(w0)
    ctx.set_warm(hsf.WARM_EXTRAP)
    nsp, T = ctx.nsp, ctx.T
    V = wls[0].V
    assert all(wl.V == V for wl in wls)
    out = {}
    rec = set(record)
    buf_phi = torch.empty(nsp * T, dtype=torch.float64, device="cuda")
    buf_w = torch.empty(nsp * T, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    for k in range(steps):
        if k in rec:
            ctx.get_densities(out=buf_phi)
        st, _ = ctx.step(1, tol=tol, max_iter=5000)
        if k in rec:
            ctx.get_fields(out=buf_w)
            out[k] = (buf_phi.view(len(wls), nsp, V).clone(), buf_w.view(len(wls), nsp, V).clone())
        if log and k % 100 == 0:
            log(f"  trajectory step {k}: iterations {[s['iterations'] for s in st]} "
                f"({time.perf_counter() - t0:.1f} s)")
    ctx.close()
    return out


def make_samples(traj, io):
    """Network samples from a recorded trajectory: for every k with k-1, k, k+1
    recorded, one first-difference and one second-difference sample per replica,
    assembled on the device by the library (hsf_net_make_sample through the network
    handle io).  Returns (x [S][2 nsp][V], y [S][2][V]) FP32 device tensors."""
    torch = _torch()
    xs, ys = [], []
    for k in sorted(traj):
        if k + 1 not in traj:
            continue
        p0, w0 = traj[k]
        p1, w1 = traj[k + 1]
        R, nsp, V = p0.shape
        prev = traj.get(k - 1)
        for mode in (1, 2):
            if mode == 2 and prev is None:
                continue
            for r in range(R):
                x = torch.empty((2 * nsp, V), dtype=torch.float32, device="cuda")
                y = torch.empty((2, V), dtype=torch.float32, device="cuda")
                io.make_sample(p1[r], p0[r], prev[0][r] if mode == 2 else None, w1[r], w0[r],
                               prev[1][r] if mode == 2 else None, nsp, V, mode, x, y)
                xs.append(x)
                ys.append(y)
    return torch.stack(xs), torch.stack(ys)


def input_norm(io, x):
    """Per-channel shift and scale of the network input: the density channels are
    standardised over the data set (moments reduced on the device), the difference
    channels already have unit rms."""
    S, C, V = x.shape
    nsp = C // 2
    mean, rms = io.channel_moments(x, S, C, V)
    shift, scale = [], []
    for c in range(C):
        if c < nsp:
            std = float(np.sqrt(max(rms[c] ** 2 - mean[c] ** 2, 0.0)))
            shift.append(float(mean[c]))
            scale.append(1.0 / max(std, 1e-6))
        else:
            shift.append(0.0)
            scale.append(1.0)
    return shift, scale


def train(net, x, y, L, iters=1500, batch=2, lr=1e-3, lr_end=1e-4, seed=0, log=None, x_val=None, y_val=None):
    """Adam on the mean square error over random mini-batches, learning rate decaying
    geometrically from lr to lr_end.  Returns the list of training losses."""
    torch = _torch()
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    S = x.shape[0]
    losses = []
    xb = torch.empty((batch,) + tuple(x.shape[1:]), dtype=torch.float32, device=x.device)
    yb = torch.empty((batch,) + tuple(y.shape[1:]), dtype=torch.float32, device=y.device)
    t0 = time.perf_counter()
    for it in range(iters):
        idx = torch.randint(0, S, (batch,), generator=g)
        xb.copy_(x[idx.to(x.device)])
        yb.copy_(y[idx.to(y.device)])
        a = lr * (lr_end / lr) ** (it / max(1, iters - 1))
        losses.append(net.train_step(xb.view(-1), yb.view(-1), batch, L, a))
        if log and (it % 250 == 0 or it == iters - 1):
            msg = f"  train iter {it}: loss {losses[-1]:.4e} lr {a:.2e} ({time.perf_counter() - t0:.1f} s)"
            if x_val is not None:
                msg += f", validation {evaluate_loss(net, x_val, y_val, L):.4e}"
            log(msg)
    return losses


def evaluate_loss(net, x, y, L, batch=2):
    tot, n = 0.0, 0
    for i in range(0, x.shape[0] - batch + 1, batch):
        l, _ = net.loss_grad(x[i:i + batch].reshape(-1), y[i:i + batch].reshape(-1), batch, L, with_grad=False)
        tot += l * batch
        n += batch
    return tot / max(n, 1)


def train_warm_start(make_workloads, seeds, steps, record, widths=DEFAULT_WIDTHS, iters=1500, batch=2, lr=1e-3,
                     lr_end=1e-4, val_seed=None, net_seed=1, log=None, precond=False, tol=1e-10):
    """Record trajectories of make_workloads(seed) for every training seed (FP64
    propagators, residual 1e-10), build the first- and second-difference samples,
    and train a network with 2 nsp inputs on them.  Returns (net, info)."""
    torch = _torch()
    t0 = time.perf_counter()
    xs, ys = [], []
    nsp = make_workloads(seeds[0])[0].nsp
    io = hsf.Net(2 * nsp, 2, (8,), seed=0)   # sample assembly and reductions
    for seed in seeds:
        traj = record_trajectory(make_workloads(seed), steps, record, tol=tol, precision="fp64", log=log,
                                 precond=precond)
        x, y = make_samples(traj, io)
        del traj
        xs.append(x)
        ys.append(y)
    x, y = torch.cat(xs), torch.cat(ys)
    del xs, ys
    t_data = time.perf_counter() - t0
    xv = yv = None
    if val_seed is not None:   # early steps of a held-out trajectory
        tv = record_trajectory(make_workloads(val_seed)[:1], 22, list(range(1, 22)), tol=tol, precision="fp64",
                               precond=precond)
        xv, yv = make_samples(tv, io)
    L = round(x.shape[2] ** (1.0 / 3.0))
    net = hsf.Net(2 * nsp, 2, widths, seed=net_seed)
    shift, scale = input_norm(io, x)
    net.set_input_norm(shift, scale)
    # targets per output channel to unit rms (the fields of a dilute species respond far
    # more strongly than the others); the scale goes back on as the network's output scale
    S, C_out, V = y.shape
    _, yr = io.channel_moments(y, S, C_out, V)
    out_rms = [max(float(v), 1e-30) for v in yr]
    inv = [1.0 / v for v in out_rms]
    io.affine(y, S, C_out, V, [0.0] * C_out, inv)
    if yv is not None:
        io.affine(yv, yv.shape[0], C_out, V, [0.0] * C_out, inv)
    io.close()
    t1 = time.perf_counter()
    losses = train(net, x, y, L, iters=iters, batch=batch, lr=lr, lr_end=lr_end, log=log, x_val=xv, y_val=yv)
    val = evaluate_loss(net, xv, yv, L) if xv is not None else None
    net.set_output_scale(out_rms)
    torch.cuda.synchronize()
    info = {"widths": list(widths), "parameters": int(net.n_params), "samples": int(x.shape[0]),
            "training_seeds": list(seeds), "iterations": iters, "batch": batch,
            "loss_first": float(losses[0]), "loss_last": float(np.mean(losses[-50:])),
            "validation_loss": val, "loss_units": "mean square error of targets scaled to unit rms per channel",
            "target_rms": out_rms,
            "data_seconds": t_data, "train_seconds": time.perf_counter() - t1}
    return net, info


def compare_warm_starts(wls, net, modes, start_steps, measure_steps, tol=1e-6, precision="fp32", tile=None,
                        log=None, gate=0, precond=False, max_iter=1000):
    """Step time and evaluations per step of each warm start on the trajectory of
    `wls`: the dynamics runs `start_steps` plain steps, the state is saved, and each
    mode then runs 2 plain steps (to build the history) and `measure_steps` timed
    steps from that same state.  Returns {mode: {...}}."""
    torch = _torch()
    ctx = hsf.Context(wls, precision=precision)
    ctx.set_solver(precond=precond)
    phi0, w0 = initial_state(ctx, wls)
    ctx.set_densities(phi0)
    ctx.set_fields(w0)
    if tile is not None:
        ctx.set_tile(tile)
    if net is not None:
        ctx.attach_net(net)
        ctx.set_net_gate(gate)
    ctx.set_warm(hsf.WARM_CURRENT)
    if start_steps:
        ctx.step(start_steps, tol=tol, max_iter=max_iter)
    snap = (ctx.get_densities(), ctx.get_fields(), ctx.get_lb())
    out = {}
    names = {hsf.WARM_CURRENT: "current", hsf.WARM_LOCAL: "local", hsf.WARM_EXTRAP: "extrapolated",
             hsf.WARM_NET: "net", hsf.WARM_NET_DELTA: "net_delta", hsf.WARM_NET_EXTRAP: "net_extrapolated"}
    for mode in modes:
        ctx.set_densities(snap[0])
        ctx.set_fields(snap[1])
        ctx.set_lb(snap[2])
        ctx.set_warm(hsf.WARM_CURRENT)
        ctx.step(2, tol=tol, max_iter=max_iter)
        ctx.set_warm(mode)
        ctx.step(1, tol=tol, max_iter=max_iter)   # warm-up of this mode's launch sequences
        evs, its, ts = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(measure_steps):
            ta = time.perf_counter()
            st, ev = ctx.step(1, tol=tol, max_iter=max_iter)
            ts.append(time.perf_counter() - ta)   # the step returns after its last status read
            evs.append(ev)
            its.append([s["iterations"] for s in st])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"ms_per_step": 1e3 * el / measure_steps, "evals_per_step": float(np.mean(evs)),
               "iterations_per_replica": float(np.mean(its)),
               "ms_median": 1e3 * float(np.median(ts)), "ms_p95": 1e3 * float(np.percentile(ts, 95))}
        out[names.get(mode, str(mode))] = res
        if log:
            log(f"  warm start {names.get(mode, mode)}: {res['ms_per_step']:.3f} ms/step, "
                f"{res['evals_per_step']:.2f} evaluations/step, {res['iterations_per_replica']:.2f} iterations")
    ctx.close()
    return out


def trajectory_arms(wls, net, arms, steps, windows, tol=1e-6, precision="fp32", tile=None, precond=False,
                    max_iter=1000, log=None, refine=False):
    """Each warm start runs the whole trajectory of `wls` from the quench for `steps`
    coupled steps (same initial state, same tiling), timing every step.  arms: list of
    (name, warm mode, gate).  windows: list of (first, last) step ranges (last
    exclusive) over which the per-step times are summarised.  refine: FP32 contexts finish
    each inversion below a residual of 1e-5 with FP64 evaluations.  Returns
    {name: {"whole": {...}, "windows": {"a-b": {...}}}} with the mean, median and 95th
    percentile step time and the mean evaluations per step of each range."""
    torch = _torch()
    out = {}
    for name, mode, gate in arms:
        ctx = hsf.Context(wls, precision=precision)
        ctx.set_solver(precond=precond, refine=refine)
        phi0, w0 = initial_state(ctx, wls)
        ctx.set_densities(phi0)
        ctx.set_fields(w0)
        if tile is not None:
            ctx.set_tile(tile)
        if net is not None:
            ctx.attach_net(net)
            ctx.set_net_gate(gate)
        ctx.set_warm(mode)
        ts = np.empty(steps)
        evs = np.empty(steps)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(steps):
            ta = time.perf_counter()
            _, ev = ctx.step(1, tol=tol, max_iter=max_iter)   # returns after its last status read
            ts[k] = time.perf_counter() - ta
            evs[k] = ev
            if log and k % 500 == 0:
                log(f"  {name}: step {k}, {1e3 * ts[k]:.2f} ms, {ev} evaluations "
                    f"({time.perf_counter() - t_start:.1f} s)")
        torch.cuda.synchronize()
        ctx.close()

        def summary(a, b):
            t = ts[a:b]
            return {"steps": int(b - a), "ms_mean": 1e3 * float(t.mean()), "ms_median": 1e3 * float(np.median(t)),
                    "ms_p95": 1e3 * float(np.percentile(t, 95)), "evals_per_step": float(evs[a:b].mean())}

        res = {"whole": summary(0, steps),
               "windows": {f"{a}-{b}": summary(a, min(b, steps)) for a, b in windows if a < steps}}
        out[name] = res
        if log:
            log(f"  {name}: whole run {res['whole']['ms_mean']:.3f} ms/step mean, "
                f"{res['whole']['evals_per_step']:.2f} evaluations/step")
    return out


# ---------------------------------------------------------------------------
# The recipe of the 128^3 vesicle benchmark: a network trained on 20 000 (phi, w) states
# of plain FP64 runs of the same chemistry at 64^3 (40 seeds x 500 steps), one
# second-difference sample per replica and step, assembled on the device by the library
# (hsf_net_make_sample) and stored in half precision (the matrix cores read bfloat16).

def record_recipe_samples(wls, steps, first, tol=1e-10, precond=True, log=None, store_dtype=None, net_io=None,
                          modes=(2,)):
    """Run the replicas `wls` (one batched FP64 context, residual tol, extrapolated warm
    start) for `steps` coupled steps and, for every step k >= first (first >= 2), build one
    sample per replica and mode from the states of steps k - 2, k - 1, k: mode 2, the
    second difference (NET_EXTRAP); mode 1, the first difference (NET_DELTA); mode 0, the
    direct map phi -> w (NET).  Returns ({mode: (X [S][C][V], Y [S][2][V])}, wall time), the
    tensors on the device in store_dtype (default float16), C = nsp in mode 0, else 2 nsp."""
    torch = _torch()
    store_dtype = store_dtype or torch.float16
    ctx = hsf.Context(wls, precision="fp64")
    ctx.set_solver(precond=precond)
    phi0, w0 = initial_state(ctx, wls)
    ctx.set_densities(phi0)
    ctx.set_fields(w0)
    ctx.set_warm(hsf.WARM_EXTRAP)
    nsp, T = ctx.nsp, ctx.T
    V = wls[0].V
    assert all(wl.V == V for wl in wls)
    R = len(wls)
    n_samples = R * max(0, steps - first)
    chans = {m: (nsp if m == 0 else 2 * nsp) for m in modes}
    store = {m: (torch.empty((n_samples, chans[m], V), dtype=store_dtype, device="cuda"),
                 torch.empty((n_samples, 2, V), dtype=store_dtype, device="cuda")) for m in modes}
    ring_phi = [torch.empty(nsp * T, dtype=torch.float64, device="cuda") for _ in range(3)]
    ring_w = [torch.empty(nsp * T, dtype=torch.float64, device="cuda") for _ in range(3)]
    bufs = {m: (torch.empty((chans[m], V), dtype=torch.float32, device="cuda"),
                torch.empty((2, V), dtype=torch.float32, device="cuda")) for m in modes}
    k_s = 0
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.get_densities(out=ring_phi[k % 3])
        st, _ = ctx.step(1, tol=tol, max_iter=5000)
        ctx.get_fields(out=ring_w[k % 3])
        if k >= first:
            a, b, c = k % 3, (k - 1) % 3, (k - 2) % 3
            for r in range(R):
                o = ctx.field_offset(r)
                sl = slice(o, o + nsp * V)
                for m in modes:
                    xb, yb = bufs[m]
                    net_io.make_sample(ring_phi[a][sl], ring_phi[b][sl] if m >= 1 else None,
                                       ring_phi[c][sl] if m == 2 else None, ring_w[a][sl],
                                       ring_w[b][sl] if m >= 1 else None, ring_w[c][sl] if m == 2 else None,
                                       nsp, V, m, xb, yb)
                    store[m][0][k_s].copy_(xb)
                    store[m][1][k_s].copy_(yb)
                k_s += 1
        if log and k % 50 == 0:
            log(f"  recipe trajectory step {k}: iterations {min(s['iterations'] for s in st)}.."
                f"{max(s['iterations'] for s in st)} ({time.perf_counter() - t0:.1f} s, {k_s} samples)")
    torch.cuda.synchronize()
    ctx.close()
    return {m: (X[:k_s], Y[:k_s]) for m, (X, Y) in store.items()}, time.perf_counter() - t0


def chunked_moments(net_io, T, chunk=64):
    """Per-channel mean and rms of a [S][C][V] tensor of any float dtype, through the
    library's reduction on float32 chunks (combined by sample count)."""
    torch = _torch()
    S, C, V = T.shape
    buf = torch.empty((min(chunk, S), C, V), dtype=torch.float32, device=T.device)
    m1 = np.zeros(C)
    m2 = np.zeros(C)
    for i in range(0, S, chunk):
        n = min(chunk, S - i)
        buf[:n].copy_(T[i:i + n])
        mean, rms = net_io.channel_moments(buf[:n], n, C, V)
        m1 += n * np.asarray(mean)
        m2 += n * np.asarray(rms) ** 2
    return m1 / S, np.sqrt(m2 / S)


def train_from_store(net, X, Y, L, iters, batch, lr, lr_end, y_scale, seed=0, log=None, Xv=None, Yv=None):
    """Adam on minibatches drawn uniformly from the stored samples; targets brought to unit
    rms per channel on the device (hsf_net_affine).  Returns the training losses and the
    validation loss (mean square error in the scaled units)."""
    torch = _torch()
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    S = X.shape[0]
    xb = torch.empty((batch,) + tuple(X.shape[1:]), dtype=torch.float32, device="cuda")
    yb = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=torch.float32, device="cuda")
    C_out, V = Y.shape[1], Y.shape[2]
    zeros = [0.0] * C_out
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        idx = torch.randint(0, S, (batch,), generator=g).to("cuda")
        xb.copy_(X[idx])
        yb.copy_(Y[idx])
        net.affine(yb, batch, C_out, V, zeros, y_scale)
        a = lr * (lr_end / lr) ** (it / max(1, iters - 1))
        losses.append(net.train_step(xb.view(-1), yb.view(-1), batch, L, a))
        if log and (it % 2000 == 0 or it == iters - 1):
            log(f"  train iter {it}: loss {np.mean(losses[-100:]):.4e} lr {a:.2e} ({time.perf_counter() - t0:.1f} s)")
    val = None
    if Xv is not None:
        tot = 0.0
        for i in range(Xv.shape[0]):
            xb[:1].copy_(Xv[i:i + 1])
            yb[:1].copy_(Yv[i:i + 1])
            net.affine(yb[:1], 1, C_out, V, zeros, y_scale)
            l, _ = net.loss_grad(xb[:1].reshape(-1), yb[:1].reshape(-1), 1, L, with_grad=False)
            tot += l
        val = tot / Xv.shape[0]
    return losses, val, time.perf_counter() - t0


def save_net(path, net, widths, in_ch, out_ch, shift, scale, out_scale, info):
    """Parameters and normalisation of a trained network (no pickled objects)."""
    import json
    np.savez(path, params=net.get_params().astype(np.float32), widths=np.asarray(widths, dtype=np.int32),
             channels=np.asarray([in_ch, out_ch], dtype=np.int32), shift=np.asarray(shift, dtype=np.float32),
             scale=np.asarray(scale, dtype=np.float32), out_scale=np.asarray(out_scale, dtype=np.float32),
             info=np.asarray(json.dumps(info)))


def load_net(path):
    """A network saved by save_net, ready for inference (output scale set).  Returns
    (net, info)."""
    import json
    z = np.load(path, allow_pickle=False)
    widths = tuple(int(v) for v in z["widths"])
    in_ch, out_ch = (int(v) for v in z["channels"])
    net = hsf.Net(in_ch, out_ch, widths, seed=0)
    net.set_params(z["params"].astype(np.float32))
    net.set_input_norm(z["shift"].tolist(), z["scale"].tolist())
    net.set_output_scale(z["out_scale"].tolist())
    return net, json.loads(str(z["info"]))


# File name of a recipe network per sample mode (2: the benchmark's NET_EXTRAP networks).
RECIPE_PREFIX = {2: "vesicle_a3b9s", 1: "vesicle_a3b9s_delta", 0: "vesicle_a3b9s_direct"}
RECIPE_SAMPLE = {2: "second difference per replica and step", 1: "first difference per replica and step",
                 0: "the state itself (phi -> w) per replica and step"}


def train_recipe(out_dir, seeds=tuple(range(1, 41)), steps=502, first=2, L=64, widths_list=((8, 16, 24, 32), (16,)),
                 iters=12000, batch=4, val_seed=99, log=None, modes=(2,)):
    """The benchmark's recipe: 40 seeds x 500 recorded steps of the A3B9 + S vesicle
    chemistry at 64^3 (20 000 (phi, w) states, FP64, residual 1e-10), one sample per
    replica, step and mode (second difference, mode 2, for the benchmark's networks; first
    difference, mode 1, and the direct map, mode 0, for the other warm starts), a held-out
    seed for validation, then each network of widths_list trained on the same samples and
    saved to out_dir.  Returns {file name: info}."""
    import os
    torch = _torch()
    os.makedirs(out_dir, exist_ok=True)
    mk = lambda seed: W.vesicle128_a3b9s(L=L).with_(seed=seed, precision="fp64")
    nsp = 3
    io = hsf.Net(2 * nsp, 2, (8,), seed=0)   # sample assembly and reductions
    data, t_data = record_recipe_samples([mk(s) for s in seeds], steps, first, log=log, net_io=io, modes=modes)
    vdata, _ = record_recipe_samples([mk(val_seed)], 40, 10, log=None, net_io=io, modes=modes)
    states = len(seeds) * (steps - first)
    results = {}
    for mode in modes:
        X, Y = data[mode]
        Xv, Yv = vdata[mode]
        cin = X.shape[1]
        if log:
            log(f"  mode {mode}: {X.shape[0]} samples from {states} states in {t_data:.1f} s")
        xm, xr = chunked_moments(io, X)
        ym, yr = chunked_moments(io, Y)
        # density channels standardised over the data; difference channels are unit rms already
        shift = [float(xm[c]) if c < nsp else 0.0 for c in range(cin)]
        scale = [1.0 / max(float(np.sqrt(max(xr[c] ** 2 - xm[c] ** 2, 0.0))), 1e-6) if c < nsp else 1.0
                 for c in range(cin)]
        out_rms = [max(float(v), 1e-30) for v in yr]
        y_scale = [1.0 / v for v in out_rms]
        for widths in widths_list:
            net = hsf.Net(cin, 2, widths, seed=1)
            net.set_input_norm(shift, scale)
            losses, val, t_train = train_from_store(net, X, Y, L, iters, batch, 1e-3, 1e-4, y_scale, log=log, Xv=Xv,
                                                    Yv=Yv)
            name = "w" + "-".join(str(w) for w in widths)
            info = {"recipe": f"{len(seeds)} seeds x {steps - first} steps of the A3B9 + S vesicle chemistry at "
                              f"{L}^3 (FP64 propagators, preconditioned inversion to 1e-10, extrapolated warm start)",
                    "states": states, "samples": int(X.shape[0]), "sample": RECIPE_SAMPLE[mode], "mode": mode,
                    "storage": "float16", "widths": list(widths), "parameters": int(net.n_params),
                    "iterations": iters, "batch": batch, "lr": [1e-3, 1e-4],
                    "loss_first": float(np.mean(losses[:50])), "loss_last": float(np.mean(losses[-500:])),
                    "validation_loss": val, "validation": f"seed {val_seed}, steps 10-39",
                    "loss_units": "mean square error of targets scaled to unit rms per channel",
                    "target_rms": out_rms, "data_seconds": t_data, "train_seconds": t_train}
            net.set_output_scale(out_rms)
            fname = f"{RECIPE_PREFIX[mode]}_{name}.npz"
            save_net(os.path.join(out_dir, fname), net, widths, cin, 2, shift, scale, out_rms, info)
            results[fname] = info
            if log:
                log(f"  network {fname}: {info}")
            net.close()
    io.close()
    return results


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="train the warm-start networks of the vesicle benchmark recipe")
    ap.add_argument("out_dir")
    ap.add_argument("--seeds", type=int, default=40)
    ap.add_argument("--steps", type=int, default=502)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--modes", default="2", help="sample modes, comma separated (2: second difference, "
                    "1: first difference, 0: direct map)")
    ap.add_argument("--widths", default="8,16,24,32;16", help="networks to train, widths separated by ';'")
    args = ap.parse_args()
    res = train_recipe(args.out_dir, seeds=tuple(range(1, args.seeds + 1)), steps=args.steps, iters=args.iters,
                       log=lambda m: print(m, file=sys.stderr, flush=True),
                       modes=tuple(int(m) for m in args.modes.split(",")),
                       widths_list=tuple(tuple(int(v) for v in w.split(",")) for w in args.widths.split(";")))
    print(json.dumps(res))
