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

Everything here runs on the GPU: the trajectories through hsf.Context, the
training through hsf.Net, the sample assembly in torch on device tensors.
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


def make_samples(traj, polymer=2):
    """Network samples from a recorded trajectory: for every k with k-1, k, k+1
    recorded, one first-difference and one second-difference sample per replica.
    Returns (x [S][2 nsp][V], y [S][2][V]) FP32 device tensors."""
    torch = _torch()
    xs, ys = [], []
    for k in sorted(traj):
        if k + 1 not in traj:
            continue
        p0, w0 = traj[k]
        p1, w1 = traj[k + 1]
        diffs = [(p1 - p0, w1 - w0)]
        if k - 1 in traj:
            pm, wm = traj[k - 1]
            diffs.append((p1 - 2 * p0 + pm, w1 - 2 * w0 + wm))
        for dp, dw in diffs:
            for r in range(p0.shape[0]):
                rms = torch.sqrt(torch.mean(dp[r] ** 2)).clamp_min(1e-300)
                xs.append(torch.cat([p0[r], dp[r] / rms]).float())
                ys.append((dw[r, :polymer] / rms).float())
    return torch.stack(xs), torch.stack(ys)


def input_norm(x):
    """Per-channel shift and scale of the network input: the density channels are
    standardised over the data set, the difference channels already have unit rms."""
    nsp = x.shape[1] // 2
    shift, scale = [], []
    for c in range(x.shape[1]):
        if c < nsp:
            m = float(x[:, c].mean())
            s = float(x[:, c].std())
            shift.append(m)
            scale.append(1.0 / max(s, 1e-6))
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
    for seed in seeds:
        traj = record_trajectory(make_workloads(seed), steps, record, tol=tol, precision="fp64", log=log,
                                 precond=precond)
        x, y = make_samples(traj)
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
        xv, yv = make_samples(tv)
    L = round(x.shape[2] ** (1.0 / 3.0))
    nsp = x.shape[1] // 2
    net = hsf.Net(2 * nsp, 2, widths, seed=net_seed)
    shift, scale = input_norm(x)
    net.set_input_norm(shift, scale)
    # targets per output channel to unit rms (the fields of a dilute species respond far
    # more strongly than the others); the scale goes back on as the network's output scale
    out_rms = [max(float(y[:, c].pow(2).mean().sqrt()), 1e-30) for c in range(y.shape[1])]
    inv = torch.tensor([1.0 / v for v in out_rms], dtype=torch.float32, device=y.device).view(1, -1, 1)
    y = y * inv
    if yv is not None:
        yv = yv * inv
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
                    max_iter=1000, log=None):
    """Each warm start runs the whole trajectory of `wls` from the quench for `steps`
    coupled steps (same initial state, same tiling), timing every step.  arms: list of
    (name, warm mode, gate).  windows: list of (first, last) step ranges (last
    exclusive) over which the per-step times are summarised.  Returns
    {name: {"whole": {...}, "windows": {"a-b": {...}}}} with the mean, median and 95th
    percentile step time and the mean evaluations per step of each range."""
    torch = _torch()
    out = {}
    for name, mode, gate in arms:
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
