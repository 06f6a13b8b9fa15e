"""Benchmark: coupled LB + dynamic-SCF steps on one GPU.

Default workload: the 64^3 periodic melt of symmetric A8B8 diblocks, chi N = 20,
initial noise +-0.01 (seed 0), at the two viscosity settings tau = 0.6 and
tau = 1.5, run together as two replicas of one batched context, propagators in
FP32 with FP64 reductions (the mixed-precision arm).  The all-FP64 arm of the
same comparison is timed after it and reported in its own field.

A step is one pass of the whole method over every replica: field inversion to
the residual, chemical potential and force, LB collide-and-stream, and the
convection-diffusion update.  The main arm starts every inversion from the
previous step's fields (the plain warm start).  The field learned_warm_start
compares, on the same workload and window, the plain, extrapolated and learned
warm starts (network trained in the same run, on other seeds).

value = propagator site-bead updates per second over the timed steps: every
density-functional evaluation performs 2 N V site-bead updates (N forward and
N backward propagator steps over V sites); the count runs over all evaluations
the inversions needed in all replicas, divided by the wall time of the steps.

Prints one JSON line.  Inputs are synthetic (seeded), resident in HBM before
the timed region starts.
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

# HBM-side bytes per launch of the dominant propagator kernel, from the counter runs
# summarised in profiles/propagator_melt64_a8b8_x2_fp32_traffic.md and
# profiles/spill_melt192_a8b8_fp32.md (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0
# after a calibration copy).  Valid only for that workload, precision, tiling and kernel
# as they stand; anything else reports null.
MEASURED_TRAFFIC = {("melt64_a8b8", "fp32", (64, 4, 2, 0), "bwd"): 13.72e6,
                    ("melt64_a8b8", "fp32", (32, 8, 2, 0), "bwd"): 13.74e6,
                    ("melt192_a8b8", "fp32", (64, 4, 8, 0), "bwd"): 185.7e6,
                    ("melt64_a8b8", "fp32", (32, 8, 2, -1), "pair"): 18.45e6}
METRIC = "propagator site·bead updates/s + LB MLUPS; step time learned vs plain at 1e-6"


def algorithmic_bytes_per_update(wl, prec_bytes):
    """Bytes per site-bead update of the store-all-G scheme: each stored G_s is
    written once and read once (prec_bytes per update), plus the polymer fields
    read once and the polymer densities written once per evaluation (FP64),
    spread over the 2N updates of the evaluation."""
    n_poly = 2
    return prec_bytes + n_poly * (8 + 8) / (2.0 * wl.N)


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


def cpu_baseline(wl, w, phi, seconds):
    from oracle import oracle as orc
    orc.build(force=False)
    sysw = orc.System(L=wl.L, types=wl.types, has_solvent=wl.has_solvent, a=wl.a, chi=wl.chi,
                      kappa=wl.kappa, dt=wl.dt, tau=wl.tau)
    pbar = phi[:2].sum(0).mean()
    pbs = phi[2].mean() if wl.has_solvent else 0.0
    n = 0
    t0 = time.perf_counter()
    while True:
        orc.evaluate(sysw, w, pbar, pbs)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    upd = n * 2 * wl.N * wl.V
    return {"value": upd / el, "unit": "site·bead updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} density-functional evaluations of the {wl.L[0]}x{wl.L[1]}x{wl.L[2]} {wl.name} system at "
                      f"the GPU run's final fields of replica 0 ({el:.1f} s, single-threaded FP64 C oracle)"}


# Recipes of the learned warm start per benchmark workload: the trajectories it is
# trained on (FP64, residual 1e-10, other seeds than the benchmark's 0), the steps
# recorded, training length, and the states (steps after the quench) where the warm
# starts are compared.
LEARNED = {
    "melt64_a8b8": dict(train=lambda W, seed: [w.with_(seed=seed) for w in make_workloads("melt64_a8b8", "fp64")],
                        seeds=(1, 2), steps=1202, iters=1500,
                        record=list(range(0, 121)) + [k for c in (300, 600, 900, 1200) for k in (c - 1, c, c + 1)],
                        later=(300, 1000)),
    # the 128^3 vesicle-forming solution, network trained on 64^3 runs of the same chemistry
    "vesicle128_a3b9s": dict(train=lambda W, seed: [W.vesicle128_a3b9s(L=64).with_(seed=seed, precision="fp64")],
                             seeds=(1, 2, 3), steps=602, iters=3000,
                             record=list(range(0, 121)) + [k for c in (300, 600) for k in (c - 1, c, c + 1)],
                             later=(200,)),
}


def learned_arm(hsf, workload, precision, steps, warmup, tile, log, precond=False, widths=None):
    """The learned warm start on the benchmark's own workload: a network trained on
    the GPU from FP64 trajectories of other seeds, then every warm start run on the
    benchmark's seed from the same states: `warmup` steps after the quench (the
    window the main arm times) and later ones.  widths: the network's level widths
    (default: the one-level net of the warm-start module)."""
    from paper_1204_2088_amd import warmnet
    from paper_1204_2088_amd import workloads as W
    rc = LEARNED[workload]
    net, info = warmnet.train_warm_start(lambda seed: rc["train"](W, seed), seeds=rc["seeds"], steps=rc["steps"],
                                         record=rc["record"], iters=rc["iters"], val_seed=5, log=None,
                                         precond=precond, widths=widths or warmnet.DEFAULT_WIDTHS)
    log(f"# warm-start network trained: {info}")
    wls = make_workloads(workload, precision)
    modes = [hsf.WARM_CURRENT, hsf.WARM_EXTRAP, hsf.WARM_NET_EXTRAP]
    regimes = {}
    for start in (warmup,) + tuple(rc["later"]):
        res = warmnet.compare_warm_starts(wls, net, modes, start, steps, tile=tile, precond=precond,
                                          log=lambda m: log(f"# [from step {start}]{m}"))
        gated = warmnet.compare_warm_starts(wls, net, [hsf.WARM_NET_EXTRAP], start, steps, tile=tile, gate=2,
                                            precond=precond, log=lambda m: log(f"# [from step {start}, gate 2]{m}"))
        res["net_extrapolated_gate2"] = gated["net_extrapolated"]
        regimes[f"from_step_{start}"] = res
    net.close()
    head = regimes[f"from_step_{warmup}"]
    return {
        "tol": wls[0].tol, "steps_per_mode": steps, "solver": "preconditioned FR" if precond else "FR",
        "window": "each mode restarts from the saved state, runs 2 plain steps and 1 untimed step of its own, "
                  "then the timed steps",
        "network": info,
        "regimes": regimes,
        "speedup_learned_vs_plain": head["current"]["ms_per_step"] / head["net_extrapolated"]["ms_per_step"],
        "speedup_learned_vs_extrapolated": head["extrapolated"]["ms_per_step"] / head["net_extrapolated"]["ms_per_step"],
    }


def run_arm(hsf, torch, wls, steps, warmup, timing, log, precond=False, tile=None, noise_omega=None, hydro=True):
    """Build a batched context, autotune, warm up, time `steps` coupled steps (with the
    LB flow, or purely diffusive with hydro=False)."""
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


def cn_arm(hsf, torch, wls, dt, steps, warmup, log, precision="fp64"):
    """Crank-Nicolson diffusion (Newton-Krylov) at a large time step on the same workload:
    simulated time per wall-clock second, to set against the explicit scheme's
    dt / ms_per_step.  FP64 propagators solve to rms(F) <= 1e-8, FP32 ones to 1e-5."""
    from paper_1204_2088_amd import workloads as W
    wls = [w.with_(precision=precision, dt=dt) for w in wls]
    ctx = hsf.Context(wls, stream=torch.cuda.current_stream())
    newton_tol = 1e-8 if precision == "fp64" else 1e-5
    ctx.set_integrator(True, tol=newton_tol, max_newton=30, krylov_dim=40)
    ctx.set_densities(torch.from_numpy(np.concatenate([W.initial_composition(w).ravel() for w in wls])).to("cuda"))
    tile, _ = ctx.autotune(reps=3)
    inv_tol = 1e-9 if precision == "fp64" else 1e-6   # first inversion; later ones start converged
    ctx.step(warmup, tol=inv_tol, max_iter=4000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = krylov = 0
    evals = 0
    for _ in range(steps):
        _, ev = ctx.step(1, tol=inv_tol, max_iter=4000)
        cs = ctx.cn_stats()
        newton += cs["newton"]
        krylov += cs["krylov"]
        evals += ev
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    f, sm, _ = ctx.observables()
    ctx.close()
    log(f"# crank-nicolson dt {dt}: {1e3 * el / steps:.2f} ms per step, {evals / steps:.1f} evaluations")
    return {"dt": dt, "steps": steps, "ms_per_step": 1e3 * el / steps, "evals_per_step": evals / steps,
            "newton_per_step": newton / steps, "krylov_per_step": krylov / steps,
            "sim_time_per_s": dt * steps / el, "propagators": precision, "newton_tol_rms": newton_tol,
            "tile": list(tile), "free_energy_end": f.tolist()[:8], "s_melt_end": sm.tolist()[:8]}


def measure_observables(ctx, torch, wl, V_total, reps=10):
    """Free-energy density and order parameters of the final state, and the cost of the
    call: each runs one evaluation (for Q) and two FP64 site passes, so the passes cost
    the difference to a plain evaluation.  Algorithmic bytes of the passes: phi and w
    once, then phi again (3 nsp doubles per site)."""
    out_dev = torch.empty(ctx.nsp * ctx.T, dtype=torch.float64, device="cuda")
    res = {}
    for name, fn in (("observables", ctx.observables), ("evaluate", lambda: ctx.evaluate(out=out_dev))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = 1e3 * (time.perf_counter() - t0) / reps
    f, sm, ss = ctx.observables()
    pass_ms = max(res["observables"] - res["evaluate"], 1e-9)
    pass_bytes = 3 * wl.nsp * 8 * V_total
    return {"free_energy": f.tolist()[:8], "s_melt": sm.tolist()[:8], "s_sol": ss.tolist()[:8],
            "ms_per_call": res["observables"], "evaluate_ms_per_call": res["evaluate"],
            "passes_ms": pass_ms, "passes_algorithmic_bytes": pass_bytes,
            "passes_gbs": pass_bytes / (pass_ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="melt64_a8b8")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--no-fp64-arm", action="store_true", help="skip the all-FP64 arm")
    ap.add_argument("--precond", action="store_true", help="diagonally preconditioned inversion")
    ap.add_argument("--tile", default=None, help="cx,cy,cz,k: use this propagator tiling instead of autotuning (k = 0: one step per launch, -1: paired forward/backward steps, >= 1: temporally blocked)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--net-widths", default=None, metavar="WIDTHS",
                    help="level widths of the learned warm start's network (e.g. 8,16,24,32; default one level of 16)")
    ap.add_argument("--lb", default="bgk", choices=["bgk", "mrt"],
                    help="LB collision: BGK, or the MRT scheme with the shear viscosity of the workload's tau, "
                         "the same bulk eigenvalue and the kinetic modes relaxed completely")
    ap.add_argument("--no-cn-arm", action="store_true", help="skip the Crank-Nicolson (dt 0.4) arm")
    ap.add_argument("--no-diffusive-arm", action="store_true",
                    help="skip the purely diffusive run (LB velocity zeroed) of the 96^3 A4B12 melt")
    ap.add_argument("--cn-dt", type=float, default=0.4, help="time step of the Crank-Nicolson arm")
    ap.add_argument("--noise", type=float, default=None, metavar="OMEGA",
                    help="thermal noise in both the compositions (eq. 5) and the LB modes (eq. 13) "
                         "with noise scaling parameter OMEGA (the paper uses 400)")
    ap.add_argument("--net-probe", default=None, metavar="WIDTHS",
                    help="only time the warm-start network of these level widths (e.g. 16 or 8,16,24,32): "
                         "forward passes and Adam steps on two 64^3 samples")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()

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

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the method is benchmarked "
              "on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_2088_amd import hsf

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    wls = make_workloads(args.workload, args.precision)
    if args.lb == "mrt":
        from paper_1204_2088_amd import workloads as W
        wls = [w.with_(lb="mrt", gammas=W.mrt_gammas(w.tau)) for w in wls]
    wl = wls[0]
    ctx, tile, tune_ms, stats, (evals, site_evals), elapsed, timing, t_steps, t_elapsed = run_arm(
        hsf, torch, wls, args.steps, args.warmup, not args.no_timing, log, args.precond,
        tuple(int(v) for v in args.tile.split(",")) if args.tile else None, args.noise)

    V_total = sum(w.V for w in wls)
    N = wl.N
    # every evaluation of every replica counts 2 N V_r site-bead updates
    updates = 2 * N * site_evals
    value = updates / elapsed
    prec_bytes = 4 if wl.precision == "fp32" else 8
    b_unit = algorithmic_bytes_per_update(wl, prec_bytes)

    roofline = None
    lb_mlups = None
    kernels = {}
    if timing:
        for k, (ms, cnt) in timing.items():
            if cnt:
                kernels[k] = {"launches": cnt, "avg_us": 1e3 * ms / cnt, "total_ms": ms}
        if "lb" in kernels:
            lb_mlups = V_total / (kernels["lb"]["avg_us"] * 1e-6) / 1e6
        prop = {k: v for k, v in kernels.items() if k in ("fwd", "bwd", "pair")}
        if prop:
            dom = max(prop, key=lambda k: prop[k]["total_ms"])
            avg_s = prop[dom]["avg_us"] * 1e-6
            # a paired launch takes forward step j and (for j < N) a backward step: 2N - 1
            # steps in N launches per evaluation
            steps_per_launch = (2 * N - 1) / N if dom == "pair" else max(1, tile[3])
            units = V_total * steps_per_launch
            achieved = b_unit * units / avg_s / 1e9
            traffic = MEASURED_TRAFFIC.get((args.workload, wl.precision, tuple(tile), dom))
            roofline = {"bound": "hbm", "kernel": f"k_{dom}", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                        "traffic_unit": "bytes per launch (counters)",
                        "algorithmic_bytes_per_launch": b_unit * units,
                        "bytes_per_update": b_unit, "updates_per_launch": units}

    observables = measure_observables(ctx, torch, wl, V_total)

    cpu = None
    if not args.no_cpu_baseline:
        nsp = wl.nsp
        w_final = ctx.get_fields()[:nsp * wl.V].reshape((nsp,) + wl.shape)
        phi_final = ctx.get_densities()[:nsp * wl.V].reshape((nsp,) + wl.shape)
        cpu = cpu_baseline(wl, w_final, phi_final, args.cpu_seconds)
    ctx.close()

    fp64_arm = None
    if args.workload.startswith("melt64_a8b8") and args.precision == "fp32" and not args.no_fp64_arm:
        wls64 = make_workloads(args.workload, "fp64")
        steps64 = max(2, args.steps // 5)
        c64, tile64, _, st64, (ev64, se64), el64, _, _, _ = run_arm(hsf, torch, wls64, steps64, 3, False, log,
                                                                   args.precond)
        fp64_arm = {"value": 2 * N * se64 / el64, "unit": "site·bead updates/s",
                    "steps": steps64, "ms_per_step": 1e3 * el64 / steps64, "evals_per_step": ev64 / steps64,
                    "tol": wls64[0].tol, "tile": list(tile64)}
        c64.close()

    cn = None
    if not args.no_cn_arm and args.workload.startswith("melt64"):
        cn = cn_arm(hsf, torch, wls, args.cn_dt, 5, 1, log)
        cn["explicit_sim_time_per_s"] = wl.dt * args.steps / elapsed
        cn["speedup_sim_time"] = cn["sim_time_per_s"] / cn["explicit_sim_time_per_s"]
        c32 = cn_arm(hsf, torch, wls, args.cn_dt, 5, 1, log, precision="fp32")
        cn["fp32"] = {k: c32[k] for k in ("ms_per_step", "evals_per_step", "newton_per_step", "krylov_per_step",
                                           "sim_time_per_s", "newton_tol_rms")}
        cn["fp32"]["speedup_sim_time"] = c32["sim_time_per_s"] / cn["explicit_sim_time_per_s"]

    diffusive = None
    if args.workload.startswith("melt96") and not args.no_diffusive_arm:
        # the asymmetric melt is run with and without the flow
        cd_, _, _, std, (evd, sed), eld, _, _, _ = run_arm(hsf, torch, wls, args.steps, args.warmup, False, log,
                                                          args.precond, tuple(tile), args.noise, hydro=False)
        diffusive = {"value": 2 * N * sed / eld, "unit": "site·bead updates/s", "steps": args.steps,
                     "ms_per_step": 1e3 * eld / args.steps, "evals_per_step": evd / args.steps,
                     "iterations_last_step": [x["iterations"] for x in std][:8], "tile": list(tile)}
        cd_.close()

    learned = None
    if args.workload in LEARNED and not args.no_learned:
        learned = learned_arm(hsf, args.workload, args.precision, args.steps, args.warmup, tuple(tile), log,
                              precond=args.precond,
                              widths=tuple(int(v) for v in args.net_widths.split(",")) if args.net_widths else None)

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
                   "tau": [w.tau for w in wls], "propagators": wl.precision, "reductions": "fp64",
                   "tol": wl.tol, "dt": wl.dt, "hydro": True,
                   "solver": "preconditioned FR" if args.precond else "FR", "lb": args.lb,
                   "noise_omega": args.noise},
        "evals_per_step": evals / args.steps,
        "iterations_last_step": [s["iterations"] for s in stats][:8],
        "lb_mlups": lb_mlups,
        "tile": {"core": list(tile[:3]), "steps_per_launch": max(1, tile[3]), "paired": tile[3] == -1, "autotune_ms_per_eval": tune_ms},
        "kernels": kernels,
        "kernel_timing_region": {"steps": t_steps,
                                 "ms_per_step": (1e3 * t_elapsed / t_steps) if t_elapsed else None,
                                 "launch": "direct, one event pair per hot kernel"},
        "roofline": roofline,
        "fp64_arm": fp64_arm,
        "diffusive_arm": diffusive,
        "learned_warm_start": learned,
        "observables": observables,
        "crank_nicolson": cn,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
