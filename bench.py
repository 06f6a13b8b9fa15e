"""Benchmark: coupled LB + dynamic-SCF steps on one GPU.

Default workload (the configuration the metric's learned-vs-plain part is quoted on):
the 128^3 vesicle-forming solution, A3B9 diblocks in a monomeric solvent at copolymer
volume fraction 0.12, chi_AB N = 25, chi_BS N = 35, chi_AS = 0, tau = 0.8, initial noise
+-0.005 (seed 0), propagators in FP32 with FP64 reductions, preconditioned
Fletcher-Reeves inversion to residual 1e-6.

A step is one pass of the whole method: field inversion to the residual, chemical
potential and force, LB collide-and-stream, and the convection-diffusion update.  The
main arm starts every inversion from the previous step's fields (the plain method).

value = propagator site-bead updates per second over the timed steps: every
density-functional evaluation performs 2 N V site-bead updates (N forward and N
backward propagator steps over V sites); the count runs over all evaluations the
inversions needed, divided by the wall time of the steps.

The JSON line also carries: the roofline of the dominant propagator kernel and of the
LB kernel (algorithmic bytes per unit of the store-all scheme, HIP-event launch times
of the same run), the FP32 error against the FP64 oracle at the run's final fields, the
FP32 inversion floor, the evaluation rate through the C ABI with device and with host
buffers (the latter including the PCIe copies), the oracle timed on one host core and on
all of them (propagator updates/s and LB MLUPS), the learned warm start against the plain and extrapolated ones
over whole trajectories, and shorter runs of the 64^3 melt pair and the 48-replica
batch.  Inputs are synthetic (seeded) and resident in HBM before the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM-side bytes per launch of the dominant propagator kernel and of the LB kernel, from the
# counter runs summarised in profiles/propagator_vesicle128_a3b9s_fp32_paired.md (FETCH_SIZE
# scaled by 2.0 and WRITE_SIZE by 1.0 after a calibration copy).
# Valid only for that workload, precision, tiling and kernel as they stand; anything
# else reports null.
MEASURED_TRAFFIC = {("vesicle128_a3b9s", "fp32", (32, 8, 4, -1), "pair"): 70.31e6,
                    ("vesicle128_a3b9s", "fp32", "lb"): 436.68e6}
METRIC = "propagator site·bead updates/s + LB MLUPS; step time learned vs plain at 1e-6"

def lb_bytes_per_site(wl):
    """Algorithmic bytes per site of the fused collide-and-stream: 19 populations read and
    19 written, the force read, density and velocity written, s bytes each: 360 B with FP64
    storage; 180 B with the FP32 storage of the FP32 contexts (the kernel's FP64 force,
    density and velocity make its own compulsory traffic 208 B, so this figure is the
    stricter one)."""
    s = 4 if wl.precision == "fp32" else 8
    return s * (2 * 19 + 3 + 4)


def bytes_per_update(wl):
    """Algorithmic bytes per site-bead update of the store-all-G scheme: each stored G_s
    is written once and read once (s bytes per update), plus one field factor per species
    read (s bytes) and one density per species written (FP64) per evaluation, spread over
    its 2N updates: s + nsp (s + 8) / (2N).  FP32: 4.75 B (64^3 A8B8 melt), 5.5 B (A3B9 + S)."""
    s = 4 if wl.precision == "fp32" else 8
    return s + wl.nsp * (s + 8) / (2.0 * wl.N)


def make_workloads(name, precision):
    from paper_1204_2088_amd import workloads as W
    if name == "melt64_a8b8":
        return [W.melt64_a8b8(tau=0.6, precision=precision), W.melt64_a8b8(tau=1.5, precision=precision)]
    if name == "melt64_a8b8_tau0.6":
        return [W.melt64_a8b8(tau=0.6, precision=precision)]
    if name == "melt16_a4b4":
        return [W.melt16_a4b4().with_(precision=precision)]
    if name == "melt192_a8b8":
        return [W.melt192_a8b8(precision=precision)]
    if name == "melt96_a4b12":
        return [W.melt96_a4b12().with_(precision=precision)]
    if name == "vesicle128_a3b9s":
        return [W.vesicle128_a3b9s().with_(precision=precision)]
    if name == "batch48_a3b9s":
        return [w.with_(precision=precision) for w in W.batch48_a3b9s()]
    raise SystemExit(f"unknown workload {name}")


def oracle_system(orc, wl):
    return orc.System(L=wl.L, types=wl.types, has_solvent=wl.has_solvent, a=wl.a, chi=wl.chi,
                      kappa=wl.kappa, dt=wl.dt, tau=wl.tau)


def cpu_baseline(wl, w, phi, seconds):
    """The FP64 oracle on the host's cores, on a bounded sample of the workload: density-
    functional evaluations at the GPU run's final fields of replica 0 (propagator
    updates/s) and LB collide-and-stream steps of the same box (MLUPS), first with the
    plain build on one core, then with its OpenMP build on all the cores it is given."""
    from oracle import oracle as orc
    orc.build(force=False)
    sysw = oracle_system(orc, wl)
    pbar = phi[:2].sum(0).mean()
    pbs = phi[2].mean() if wl.has_solvent else 0.0
    n0 = orc.lb_rest_state(sysw)
    rng = np.random.Generator(np.random.PCG64(7))
    n0 = n0 * (1.0 + 0.01 * rng.uniform(-1, 1, size=n0.shape))
    f = 1e-4 * rng.uniform(-1, 1, size=(3,) + wl.shape)
    out = {}
    for label, par in (("one_core", False), ("all_cores", True)):
        threads = orc.set_parallel(par)
        budget = seconds * (0.7 if not par else 0.35)
        n, t0 = 0, time.perf_counter()
        while True:
            orc.evaluate(sysw, w, pbar, pbs)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                break
        lb_n, t1 = 0, time.perf_counter()
        nn = n0
        while True:
            nn, _, _ = orc.lb_step(sysw, nn, f)
            lb_n += 1
            el_lb = time.perf_counter() - t1
            if el_lb >= budget / 3:
                break
        out[label] = {"threads": threads, "evaluations": n, "seconds": el,
                      "updates_per_s": n * 2 * wl.N * wl.V / el,
                      "lb_steps": lb_n, "lb_seconds": el_lb, "lb_mlups": lb_n * wl.V / el_lb / 1e6,
                      "ms_per_evaluation": 1e3 * el / n}
    orc.set_parallel(False)
    one, allc = out["one_core"], out["all_cores"]
    return {"value": one["updates_per_s"], "unit": "site·bead updates/s", "cores": 1, "kind": "oracle",
            "nproc": os.cpu_count(), "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "all_cores": {"value": allc["updates_per_s"], "threads": allc["threads"],
                          "lb_mlups": allc["lb_mlups"], "ms_per_evaluation": allc["ms_per_evaluation"]},
            "lb_mlups_one_core": one["lb_mlups"], "ms_per_evaluation_one_core": one["ms_per_evaluation"],
            "sample": f"{one['evaluations']} (one core) and {allc['evaluations']} ({allc['threads']} threads) "
                      f"density-functional evaluations of the {wl.L[0]}x{wl.L[1]}x{wl.L[2]} {wl.name} system at "
                      f"the GPU run's final fields of replica 0, and {one['lb_steps']} / {allc['lb_steps']} LB "
                      f"steps of the same box (FP64 C oracle; OpenMP over z-planes for all cores)",
            "detail": out}


def oracle_error(ctx, wl, orc_threads=True):
    """Densities of the GPU evaluation at the run's final fields against the FP64 oracle's
    at the same fields (replica 0): max |difference| / max |oracle| per species."""
    from oracle import oracle as orc
    orc.build(force=False)
    nsp, V = wl.nsp, wl.V
    w = ctx.get_fields()[:nsp * V].reshape((nsp,) + wl.shape)
    phi = ctx.get_densities()[:nsp * V].reshape((nsp,) + wl.shape)
    got, q = ctx.evaluate()
    got = got[:nsp * V].reshape((nsp,) + wl.shape)
    orc.set_parallel(orc_threads)
    ref, qref = orc.evaluate(oracle_system(orc, wl), w, phi[:2].sum(0).mean(),
                             phi[2].mean() if wl.has_solvent else 0.0)
    orc.set_parallel(False)
    errs = [float(np.max(np.abs(got[I] - ref[I])) / np.max(np.abs(ref[I]))) for I in range(nsp)]
    return {"max_rel_per_species": errs, "max_rel": max(errs), "q_rel": abs(q[0] / qref - 1.0),
            "at": "final fields of the timed run, replica 0", "bound": 1e-5 if wl.precision == "fp32" else 1e-10}


def inversion_floor(ctx, wls, precond):
    """Smallest residual the inversion reaches at the run's final densities: from its
    converged fields, iterate toward tolerance 1e-14 for a bounded number of iterations."""
    from paper_1204_2088_amd import hsf
    w0 = ctx.get_fields()
    st, rc = ctx.invert(tol=1e-14, max_iter=400, warm=hsf.WARM_CURRENT, allow_noconv=True)
    out = {"residual_reached": [s["residual"] for s in st][:8], "iterations": [s["iterations"] for s in st][:8],
           "max_iter": 400, "tol_requested": 1e-14, "solver": "preconditioned FR" if precond else "FR"}
    if wls[0].precision == "fp32":
        # the same from the same fields with FP64 refinement (FP32 evaluations to 1e-5, then FP64)
        ctx.set_fields(w0)
        ctx.set_solver(precond=precond, refine=True)
        st, rc = ctx.invert(tol=1e-10, max_iter=400, warm=hsf.WARM_CURRENT, allow_noconv=True)
        ctx.set_solver(precond=precond, refine=False)
        out["refined"] = {"tol_requested": 1e-10, "residual_reached": [s["residual"] for s in st][:8],
                          "iterations": [s["iterations"] for s in st][:8],
                          "evaluations": [s["evaluations"] for s in st][:8], "converged": rc == hsf.HSF_OK}
    return out


# Recipes of the learned warm start per benchmark workload: the trajectories it is
# trained on (FP64, residual 1e-10, other seeds than the benchmark's 0), the steps
# recorded and the training length.
LEARNED = {
    "melt64_a8b8": dict(train=lambda W, seed: [w.with_(seed=seed) for w in make_workloads("melt64_a8b8", "fp64")],
                        seeds=(1, 2), steps=1202, iters=1500,
                        record=list(range(0, 121)) + [k for c in (300, 600, 900, 1200) for k in (c - 1, c, c + 1)]),
    # the 128^3 vesicle-forming solution, network trained on 64^3 runs of the same chemistry
    "vesicle128_a3b9s": dict(train=lambda W, seed: [W.vesicle128_a3b9s(L=64).with_(seed=seed, precision="fp64")],
                             seeds=(1, 2, 3), steps=602, iters=3000,
                             record=list(range(0, 121)) + [k for c in (300, 600) for k in (c - 1, c, c + 1)]),
}


# Networks trained by the vesicle recipe (python -m paper_1204_2088_amd.warmnet DIR: 40 seeds x
# 500 steps of the same chemistry at 64^3), shipped with the package.
RECIPE_NETS = {"vesicle128_a3b9s": ["vesicle_a3b9s_w8-16-24-32.npz", "vesicle_a3b9s_w16.npz"]}
# The other learned warm starts of the same recipe (--extra-arms): the first-difference
# network (NET_DELTA) and the direct map phi -> w (NET).
RECIPE_EXTRA = {"vesicle128_a3b9s": [("delta", "vesicle_a3b9s_delta_w16.npz", "WARM_NET_DELTA"),
                                     ("direct", "vesicle_a3b9s_direct_w16.npz", "WARM_NET")]}


def learned_arm(hsf, workload, precision, steps, tile, log, precond=False, widths=None, extra=False, refine=False):
    """The learned warm start on the benchmark's own workload: the recipe's networks
    (trained on the GPU from FP64 trajectories of other seeds, loaded from the package), or
    a network trained in this run when they are absent; then the cold (local guess), plain
    (previous fields), extrapolated and learned warm starts (with and without the gate) each
    run the benchmark's whole trajectory from the quench (seed 0, same tiling), every step
    timed."""
    from paper_1204_2088_amd import warmnet
    from paper_1204_2088_amd import workloads as W
    nets, infos = {}, {}
    for fname in RECIPE_NETS.get(workload, []):
        path = os.path.join(ROOT, "paper_1204_2088_amd", "nets", fname)
        if os.path.exists(path) and not widths:
            net, info = warmnet.load_net(path)
            name = fname.split("_")[-1].replace(".npz", "")
            nets[name], infos[name] = net, dict(info, file=f"paper_1204_2088_amd/nets/{fname}")
    if not nets:
        rc = LEARNED[workload]
        t0 = time.perf_counter()
        net, info = warmnet.train_warm_start(lambda seed: rc["train"](W, seed), seeds=rc["seeds"], steps=rc["steps"],
                                             record=rc["record"], iters=rc["iters"], val_seed=5, log=None,
                                             precond=precond, widths=widths or warmnet.DEFAULT_WIDTHS)
        info["wall_seconds"] = time.perf_counter() - t0
        name = "w" + "-".join(str(w) for w in (widths or warmnet.DEFAULT_WIDTHS))
        nets[name], infos[name] = net, dict(info, file="trained in this run")
    log(f"# warm-start networks: {infos}")
    wls = make_workloads(workload, precision)
    cold_steps = min(steps, 300)
    windows = [(0, 100), (100, 1000), (1000, 3000), (0, cold_steps)]
    # cold: every inversion from the local ideal-gas guess w_I = -ln phi_I (no memory of the
    # previous step; about 25 times slower per step, so it runs the first cold_steps steps
    # only); plain: the previous step's fields; extrapolated: 2 w^n - w^(n-1)
    res = warmnet.trajectory_arms(wls, None, [("cold", hsf.WARM_LOCAL, 0)], cold_steps,
                                  [(0, 100), (100, cold_steps), (0, cold_steps)], tol=wls[0].tol,
                                  precision=precision, tile=tile, precond=precond, log=log, refine=refine)
    base = [("plain", hsf.WARM_CURRENT, 0), ("extrapolated", hsf.WARM_EXTRAP, 0)]
    res.update(warmnet.trajectory_arms(wls, None, base, steps, windows, tol=wls[0].tol, precision=precision,
                                       tile=tile, precond=precond, log=log, refine=refine))
    learned_names = []
    for name, net in nets.items():
        arms = [(f"learned_{name}", hsf.WARM_NET_EXTRAP, 0), (f"learned_{name}_gate2", hsf.WARM_NET_EXTRAP, 2)]
        res.update(warmnet.trajectory_arms(wls, net, arms, steps, windows, tol=wls[0].tol, precision=precision,
                                           tile=tile, precond=precond, log=log, refine=refine))
        learned_names += [a[0] for a in arms]
        net.close()
    if extra:
        for tag, fname, mode in RECIPE_EXTRA.get(workload, []):
            path = os.path.join(ROOT, "paper_1204_2088_amd", "nets", fname)
            if not os.path.exists(path):
                continue
            net, info = warmnet.load_net(path)
            infos[f"{tag}_w16"] = dict(info, file=f"paper_1204_2088_amd/nets/{fname}")
            arms = [(f"learned_{tag}_w16", getattr(hsf, mode), 0)]
            res.update(warmnet.trajectory_arms(wls, net, arms, steps, windows, tol=wls[0].tol, precision=precision,
                                               tile=tile, precond=precond, log=log, refine=refine))
            learned_names += [a[0] for a in arms]
            net.close()
    best_learned = min(learned_names, key=lambda k: res[k]["whole"]["ms_mean"])
    best_plain = min(("plain", "extrapolated"), key=lambda k: res[k]["whole"]["ms_mean"])
    ml = res[best_learned]["whole"]["ms_mean"]
    return {
        "tol": wls[0].tol, "steps": steps,
        "solver": ("preconditioned FR" if precond else "FR") + (", FP64 evaluations below 1e-5" if refine else ""),
        "protocol": "each warm start runs the whole trajectory from the quench (seed 0), every step timed "
                    "(the cold start its first cold_steps steps, compared with the same steps of the best "
                    "learned arm); windows are step ranges of that trajectory; gate2: the network is used "
                    "only after an inversion of at least 2 iterations, else the extrapolation",
        "networks": infos,
        "arms": res,
        "best_learned_arm": best_learned,
        "best_non_learned_arm": best_plain,
        "speedup_learned_vs_cold": res["cold"]["whole"]["ms_mean"]
        / res[best_learned]["windows"][f"0-{cold_steps}"]["ms_mean"],
        "cold_steps": cold_steps,
        "speedup_learned_vs_plain": res["plain"]["whole"]["ms_mean"] / ml,
        "speedup_learned_vs_extrapolated": res["extrapolated"]["whole"]["ms_mean"] / ml,
        "speedup_learned_vs_best_non_learned": res[best_plain]["whole"]["ms_mean"] / ml,
    }


def boundary_rates(ctx, torch, wl, reps=20):
    """Evaluation rate through the C ABI with the fields set and the densities read back
    on each call, the buffers on the device (what `value` assumes: inputs resident in HBM)
    or on the host (pageable numpy arrays, or pinned torch tensors), so the host rate
    includes the PCIe copies of w in and phi out (FP64, n_species x V each)."""
    n = ctx.nsp * ctx.T
    w_dev = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.get_fields(out=w_dev)
    out_dev = torch.empty(n, dtype=torch.float64, device="cuda")
    w_np = w_dev.cpu().numpy().copy()
    out_np = np.empty(n)
    w_pin = torch.empty(n, dtype=torch.float64, pin_memory=True)
    w_pin.copy_(torch.from_numpy(w_np))
    out_pin = torch.empty(n, dtype=torch.float64, pin_memory=True)
    cases = {"device": (w_dev, out_dev), "host_pageable": (w_np, out_np), "host_pinned": (w_pin, out_pin)}
    upd = 2 * wl.N * ctx.T
    res = {}
    for name, (w, o) in cases.items():
        for _ in range(3):
            ctx.set_fields(w)
            ctx.evaluate(o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.set_fields(w)
            ctx.evaluate(o)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        res[name] = {"ms_per_call": 1e3 * el, "updates_per_s": upd / el}
    res["bytes_per_call"] = 2 * 8 * n
    res["calls"] = reps
    return res


def run_arm(hsf, torch, wls, steps, warmup, timing, log, precond=False, tile=None, noise_omega=None, hydro=True):
    """Build a batched context, autotune, warm up, time `steps` coupled steps (with the
    LB flow, or purely diffusive with hydro=False), then (timing) half as many steps with
    every hot kernel bracketed by HIP events."""
    from paper_1204_2088_amd import workloads as W
    stream = torch.cuda.current_stream()
    ctx = hsf.Context(wls, stream=stream)
    ctx.set_solver(precond=precond)
    ctx.set_hydro(hydro)
    if noise_omega:
        ctx.set_noise(cd=True, lb=True, omega=noise_omega, seed=2012)
    phi0 = np.concatenate([W.initial_composition(w).ravel() for w in wls])
    ctx.set_densities(torch.from_numpy(phi0).to("cuda"))
    torch.cuda.synchronize()
    if tile is None:
        tile, tune_ms = ctx.autotune(reps=5)
        log(f"# {wls[0].name} x{len(wls)} {wls[0].precision}: autotuned tile {tile} ({tune_ms:.3f} ms per evaluation)")
    else:
        ctx.set_tile(tile)
        tile, tune_ms = ctx.get_tile(), None
        log(f"# {wls[0].name} x{len(wls)} {wls[0].precision}: tile {tile} (given)")
    tol = wls[0].tol
    ctx.step(warmup, tol=tol, max_iter=4000)   # also captures the launch graphs
    torch.cuda.synchronize()
    ctx.get_work(reset=True)
    t0 = time.perf_counter()
    stats, evals = ctx.step(steps, tol=tol, max_iter=4000)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _, site_evals = ctx.get_work(reset=True)
    log(f"# timed {steps} steps in {elapsed:.3f} s, {evals} evaluations")
    timing_out = {}
    t_elapsed = None
    t_steps = 0
    if timing:
        # kernel-timing region: the same run continued with every hot kernel launched
        # directly and bracketed by HIP events (hipExtLaunchKernelGGL) on its stream
        t_steps = max(1, steps // 2)
        ctx.set_timing(True)
        ctx.get_timing()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.step(t_steps, tol=tol, max_iter=4000)
        torch.cuda.synchronize()
        t_elapsed = time.perf_counter() - ta
        timing_out = ctx.get_timing()
        ctx.set_timing(False)
    return ctx, tile, tune_ms, stats, (evals, site_evals), elapsed, timing_out, t_steps, t_elapsed


def rooflines(timing, wls, tile, workload):
    """Per-kernel event times, and the rooflines of the dominant propagator kernel and of
    the LB kernel: achieved = algorithmic bytes per launch / average launch time."""
    wl = wls[0]
    V_total = sum(w.V for w in wls)
    N = wl.N
    kernels = {}
    for k, (ms, cnt) in timing.items():
        if cnt:
            kernels[k] = {"launches": cnt, "avg_us": 1e3 * ms / cnt, "total_ms": ms}
    prop_roof = lb_roof = None
    prop = {k: v for k, v in kernels.items() if k in ("fwd", "bwd", "pair")}
    if prop:
        dom = max(prop, key=lambda k: prop[k]["total_ms"])
        avg_s = prop[dom]["avg_us"] * 1e-6
        # a paired launch takes forward step j and (for j < N) a backward step: 2N - 1 steps
        # in N launches per evaluation
        steps_per_launch = (2 * N - 1) / N if dom == "pair" else max(1, tile[3])
        units = V_total * steps_per_launch
        b_unit = bytes_per_update(wl)
        achieved = b_unit * units / avg_s / 1e9
        traffic = MEASURED_TRAFFIC.get((workload, wl.precision, tuple(tile), dom))
        prop_roof = {"bound": "hbm", "kernel": f"k_{dom}", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (counters)",
                     "traffic_frac": traffic / avg_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "algorithmic_bytes_per_launch": b_unit * units,
                     "bytes_per_update": b_unit, "updates_per_launch": units, "avg_launch_us": prop[dom]["avg_us"]}
    if "lb" in kernels:
        avg_s = kernels["lb"]["avg_us"] * 1e-6
        lb_b = lb_bytes_per_site(wl)
        achieved = lb_b * V_total / avg_s / 1e9
        lb_traffic = MEASURED_TRAFFIC.get((workload, wl.precision, "lb"))
        lb_roof = {"bound": "hbm", "kernel": "k_lb", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": achieved / HBM_PEAK_GBS, "bytes_per_site": lb_b,
                   "traffic": lb_traffic, "traffic_unit": "bytes per launch (counters)",
                   "traffic_frac": lb_traffic / avg_s / 1e9 / HBM_PEAK_GBS if lb_traffic else None,
                   "storage": "fp32 deviations from the rest state" if wl.precision == "fp32" else "fp64",
                   "mlups": V_total / avg_s / 1e6, "avg_launch_us": kernels["lb"]["avg_us"]}
    return kernels, prop_roof, lb_roof


def drift_arm(hsf, torch, steps, log):
    """The 64^3 A8B8 melt pair (tau 0.6 and 1.5) run twice from the same quench, with FP32
    propagators (residual 1e-6) and with FP64 ones (residual 1e-8): after every step, the
    largest density difference between the two trajectories on the 32^3 crop [0, 32)^3, per
    replica, relative to the largest FP64 density there."""
    from paper_1204_2088_amd import workloads as W
    runs = {}
    for prec in ("fp32", "fp64"):
        wls = make_workloads("melt64_a8b8", prec)
        ctx = hsf.Context(wls, stream=torch.cuda.current_stream())
        ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
        ctx.autotune(reps=2)
        runs[prec] = (ctx, wls[0].tol)
    wl = make_workloads("melt64_a8b8", "fp64")[0]
    V, shp = wl.V, (2,) + wl.shape
    err = np.zeros((steps, 2))
    t0 = time.perf_counter()
    for k in range(steps):
        phis = {}
        for prec, (ctx, tol) in runs.items():
            ctx.step(1, tol=tol, max_iter=4000)
            phis[prec] = ctx.get_densities()
        for r in range(2):
            a = phis["fp32"][2 * V * r:2 * V * (r + 1)].reshape(shp)[:, :32, :32, :32]
            b = phis["fp64"][2 * V * r:2 * V * (r + 1)].reshape(shp)[:, :32, :32, :32]
            err[k, r] = np.max(np.abs(a - b)) / np.max(np.abs(b))
        if k % 500 == 0:
            log(f"# drift step {k}: {err[k].tolist()} ({time.perf_counter() - t0:.1f} s)")
    for ctx, _ in runs.values():
        ctx.close()
    marks = [s for s in (1, 10, 100, 500, 1000, 1500, 2000) if s <= steps]
    return {"steps": steps, "crop": "[0, 32)^3", "replicas": "tau 0.6, tau 1.5",
            "max": err.max(axis=0).tolist(), "at_step": {str(m): err[m - 1].tolist() for m in marks},
            "argmax_step": (err.argmax(axis=0) + 1).tolist()}


def short_run(hsf, torch, name, steps, warmup, log, precond):
    """A shorter run of another configuration: throughput, step time and rooflines."""
    wls = make_workloads(name, "fp32")
    ctx, tile, _, _, (ev, se), el, timing, _, _ = run_arm(hsf, torch, wls, steps, warmup, True, log, precond)
    kernels, roof, lb = rooflines(timing, wls, tile, name)
    ctx.close()
    return {"workload": name, "replicas": len(wls), "sites": sum(w.V for w in wls), "steps": steps,
            "value": 2 * wls[0].N * se / el, "unit": "site·bead updates/s", "ms_per_step": 1e3 * el / steps,
            "evals_per_step": ev / steps, "tile": list(tile), "solver": "preconditioned FR" if precond else "FR",
            "roofline": roof, "lb_roofline": lb}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="vesicle128_a3b9s")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU work of the oracle baseline (split over one core and all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--precond", default="auto", choices=["auto", "on", "off"],
                    help="diagonally preconditioned inversion (auto: on for solutions)")
    ap.add_argument("--tile", default=None, help="cx,cy,cz,k: use this propagator tiling instead of autotuning (k = 0: one step per launch, -1: paired forward/backward steps, >= 1: temporally blocked)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--arms-refine", action="store_true",
                    help="run the warm-start arms with FP64 evaluations below a residual of 1e-5 (their "
                         "evaluation counts then no longer depend on FP32 rounding near the inversion floor)")
    ap.add_argument("--extra-arms", action="store_true",
                    help="also run the NET_DELTA and NET warm starts of the recipe (first-difference and direct-map "
                         "networks) over the same trajectory")
    ap.add_argument("--compare-steps", type=int, default=3000,
                    help="trajectory length of each warm start in the learned comparison")
    ap.add_argument("--net-widths", default=None, metavar="WIDTHS",
                    help="level widths of the learned warm start's network (e.g. 8,16,24,32; default one level of 16)")
    ap.add_argument("--no-extra", action="store_true", help="skip the 64^3 melt pair and the 48-replica batch")
    ap.add_argument("--lean", action="store_true",
                    help="only the main arm (for profiler runs): no oracle comparison, inversion floor, CPU "
                         "baseline, learned comparison or other configurations")
    ap.add_argument("--lb", default="bgk", choices=["bgk", "mrt"],
                    help="LB collision: BGK, or the MRT scheme with the shear viscosity of the workload's tau, "
                         "the same bulk eigenvalue and the kinetic modes relaxed completely")
    ap.add_argument("--noise", type=float, default=None, metavar="OMEGA",
                    help="thermal noise in both the compositions (eq. 5) and the LB modes (eq. 13) "
                         "with noise scaling parameter OMEGA (the paper uses 400)")
    ap.add_argument("--drift-steps", type=int, default=0,
                    help="only compare FP32 and FP64 trajectories of the 64^3 melt pair over this many steps")
    ap.add_argument("--cn-arm", action="store_true", help="also time Crank-Nicolson steps (dt --cn-dt)")
    ap.add_argument("--cn-dt", type=float, default=0.4, help="time step of the Crank-Nicolson arm")
    ap.add_argument("--net-probe", default=None, metavar="WIDTHS",
                    help="only time the warm-start network of these level widths (e.g. 16 or 8,16,24,32): "
                         "forward passes and Adam steps on two 64^3 samples")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.lean:
        args.no_cpu_baseline = args.no_learned = args.no_extra = True

    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 5}))
        return

    if args.net_probe:
        import torch
        from paper_1204_2088_amd import hsf
        widths = tuple(int(v) for v in args.net_probe.split(","))
        net = hsf.Net(4, 2, widths, seed=1)
        B, L = 2, 64
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        x = torch.rand(B * 4 * L ** 3, dtype=torch.float32, device="cuda", generator=g)
        t = torch.rand(B * 2 * L ** 3, dtype=torch.float32, device="cuda", generator=g)
        y = torch.empty_like(t)
        out = {"net_probe": list(widths), "parameters": int(net.n_params), "batch": B, "L": L}
        for name, fn, reps in (("forward", lambda: net.forward(x, B, L, out=y), 20),
                               ("train_step", lambda: net.train_step(x, t, B, L, 1e-4), 10)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            out[f"{name}_ms"] = 1e3 * (time.perf_counter() - t0) / reps
        print(json.dumps(out))
        return

    if args.drift_steps:
        import torch
        from paper_1204_2088_amd import hsf
        torch.cuda.set_device(0)
        print(json.dumps({"fp32_vs_fp64_trajectory": drift_arm(hsf, torch, args.drift_steps,
                                                               lambda m: print(m, file=sys.stderr, flush=True))}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the method is benchmarked "
              "on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_2088_amd import hsf

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t_job = time.perf_counter()
    torch.cuda.set_device(0)
    wls = make_workloads(args.workload, args.precision)
    if args.lb == "mrt":
        from paper_1204_2088_amd import workloads as W
        wls = [w.with_(lb="mrt", gammas=W.mrt_gammas(w.tau)) for w in wls]
    wl = wls[0]
    precond = wl.has_solvent if args.precond == "auto" else args.precond == "on"
    ctx, tile, tune_ms, stats, (evals, site_evals), elapsed, timing, t_steps, t_elapsed = run_arm(
        hsf, torch, wls, args.steps, args.warmup, not args.no_timing, log, precond,
        tuple(int(v) for v in args.tile.split(",")) if args.tile else None, args.noise)

    V_total = sum(w.V for w in wls)
    N = wl.N
    # every evaluation of every replica counts 2 N V_r site-bead updates
    value = 2 * N * site_evals / elapsed
    kernels, roofline, lb_roofline = rooflines(timing, wls, tile, args.workload) if timing else ({}, None, None)

    err = floor = boundary = None
    if not args.lean:
        err = oracle_error(ctx, wl)
        log(f"# error against the oracle at the final fields: {err['max_rel']:.2e}")
        floor = inversion_floor(ctx, wls, precond)
        log(f"# inversion floor: {floor['residual_reached']}; with FP64 refinement: "
            f"{floor.get('refined', {}).get('residual_reached')}")
        boundary = boundary_rates(ctx, torch, wl)
        log("# evaluation through the ABI: " + ", ".join(
            f"{k} {v['ms_per_call']:.3f} ms" for k, v in boundary.items() if isinstance(v, dict)))

    cpu = None
    if not args.no_cpu_baseline:
        nsp = wl.nsp
        w_final = ctx.get_fields()[:nsp * wl.V].reshape((nsp,) + wl.shape)
        phi_final = ctx.get_densities()[:nsp * wl.V].reshape((nsp,) + wl.shape)
        cpu = cpu_baseline(wl, w_final, phi_final, args.cpu_seconds)
        log(f"# cpu baseline: {cpu['value']:.3e} (1 core), {cpu['all_cores']['value']:.3e} "
            f"({cpu['all_cores']['threads']} threads) updates/s")
    ctx.close()

    learned = None
    if args.workload in LEARNED and not args.no_learned:
        learned = learned_arm(hsf, args.workload, args.precision, args.compare_steps, tuple(tile), log,
                              precond=precond,
                              widths=tuple(int(v) for v in args.net_widths.split(",")) if args.net_widths else None,
                              extra=args.extra_arms, refine=args.arms_refine)

    extra = {}
    if not args.no_extra and args.workload == "vesicle128_a3b9s":
        extra["melt64_a8b8"] = short_run(hsf, torch, "melt64_a8b8", 20, 5, log, False)
        extra["batch48_a3b9s"] = short_run(hsf, torch, "batch48_a3b9s", 4, 2, log, True)

    cn = None
    if args.cn_arm:
        from paper_1204_2088_amd import workloads as W
        cwls = [w.with_(precision="fp64", dt=args.cn_dt) for w in wls]
        c = hsf.Context(cwls, stream=torch.cuda.current_stream())
        c.set_integrator(True, tol=1e-8, max_newton=30, krylov_dim=40)
        c.set_densities(torch.from_numpy(np.concatenate([W.initial_composition(w).ravel() for w in cwls])).to("cuda"))
        c.autotune(reps=3)
        c.step(1, tol=1e-9, max_iter=4000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ev = c.step(5, tol=1e-9, max_iter=4000)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        c.close()
        cn = {"dt": args.cn_dt, "steps": 5, "ms_per_step": 1e3 * el / 5, "evals_per_step": ev / 5,
              "sim_time_per_s": args.cn_dt * 5 / el, "explicit_sim_time_per_s": wl.dt * args.steps / elapsed}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site·bead updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": list(wl.L), "N": N, "replicas": len(wls),
                   "species": wl.nsp, "phi_p": wl.phi_p, "tau": [w.tau for w in wls][:4],
                   "propagators": wl.precision, "reductions": "fp64", "tol": wl.tol, "dt": wl.dt, "hydro": True,
                   "solver": "preconditioned FR" if precond else "FR", "warm_start": "previous step's fields",
                   "lb": args.lb, "noise_omega": args.noise},
        "evals_per_step": evals / args.steps,
        "iterations_last_step": [s["iterations"] for s in stats][:8],
        "lb_mlups": lb_roofline["mlups"] if lb_roofline else None,
        "tile": {"core": list(tile[:3]), "steps_per_launch": max(1, tile[3]), "paired": tile[3] == -1,
                 "autotune_ms_per_eval": tune_ms},
        "kernels": kernels,
        "kernel_timing_region": {"steps": t_steps,
                                 "ms_per_step": (1e3 * t_elapsed / t_steps) if t_elapsed else None,
                                 "launch": "direct, one event pair per hot kernel"},
        "roofline": roofline,
        "lb_roofline": lb_roofline,
        "error_vs_oracle": err,
        "inversion_floor": floor,
        "host_boundary": boundary,
        "learned_warm_start": learned,
        "other_configs": extra or None,
        "crank_nicolson": cn,
        "cpu_baseline": cpu,
        "job_seconds": time.perf_counter() - t_job,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
