"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration the benchmark times (autotuned tiling, batched replicas): one
density-functional evaluation compared with the FP64 oracle at every site, and the
FP32 path's error along a trajectory of the 64^3 melt on the 32^3 crop [0, 32)^3.

Tolerances as in test_gpu_parity: 1e-5 relative for FP32 propagators, 1e-10 for FP64
(max |difference| / max |oracle value| per species).
"""
import sys

import numpy as np
import pytest

from paper_1204_2088_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def hsf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1204_2088_amd import hsf as H
    H.load()
    return H


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def osys(orc, wl):
    return orc.System(L=wl.L, types=wl.types, has_solvent=wl.has_solvent, a=wl.a, chi=wl.chi,
                      kappa=wl.kappa, dt=wl.dt, tau=wl.tau, hydro=wl.hydro)


def relerr(a, b):
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return max(np.max(np.abs(a[i] - b[i])) / np.max(np.abs(b[i])) for i in range(b.shape[0]))


def structured_fields(wl, seed):
    """Smooth fields with the amplitude of a segregating system."""
    return np.ascontiguousarray(W.random_fields((wl.nsp,) + wl.shape, seed=seed, amplitude=1.5, smooth=3))


def check_context(hsf, orc, wls, ctx, replicas, tol):
    """Evaluate the context's current fields and compare the given replicas with the oracle."""
    got, q = ctx.evaluate()
    for r in replicas:
        wl = wls[r]
        fo = ctx.field_offset(r)
        n = wl.nsp * wl.V
        w = ctx.get_fields()[fo:fo + n].reshape((wl.nsp,) + wl.shape)
        phi = ctx.get_densities()[fo:fo + n].reshape((wl.nsp,) + wl.shape)
        pbar = phi[:2].sum(0).mean()
        pbs = phi[2].mean() if wl.has_solvent else 0.0
        ref, qref = orc.evaluate(osys(orc, wl), w, pbar, pbs)
        e = relerr(got[fo:fo + n], ref)
        say(f"  replica {r} {wl.name} L={wl.L}: rel err {e:.3e}, Q {q[r]:.6e} vs {qref:.6e}")
        assert e < tol and abs(q[r] / qref - 1) < tol, (r, e)


@pytest.mark.parametrize("name", ["melt64_a8b8_pair", "melt96_a4b12", "vesicle128_a3b9s"])
def test_full_size_evaluation(hsf, orc, name):
    if name == "melt64_a8b8_pair":
        wls = [W.melt64_a8b8(tau=0.6), W.melt64_a8b8(tau=1.5)]
    elif name == "melt96_a4b12":
        wls = [W.melt96_a4b12()]
    else:
        wls = [W.vesicle128_a3b9s()]
    say(f"[full size {name}]")
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    ctx.set_fields(np.concatenate([structured_fields(w, seed=20 + r).ravel() for r, w in enumerate(wls)]))
    tile, ms = ctx.autotune(reps=2)
    say(f"  autotuned tile {tile} ({ms:.3f} ms per evaluation)")
    check_context(hsf, orc, wls, ctx, range(len(wls)), TOL32)
    ctx.close()


def test_full_size_batch48_all_replicas(hsf, orc):
    """The 48 uneven replicas in one context (preconditioned inversion, autotuned tiling,
    LB flow on) after three coupled steps from the quench: one evaluation at the run's own
    fields, every replica compared with the oracle at every site (the oracle's OpenMP
    build, bit-identical to the plain one)."""
    wls = W.batch48_a3b9s()
    say("[full size batch48_a3b9s, every replica]")
    ctx = hsf.Context(wls)
    ctx.set_solver(precond=True)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    tile, ms = ctx.autotune(reps=2)
    say(f"  autotuned tile {tile} ({ms:.3f} ms per evaluation)")
    st, _ = ctx.step(3, tol=1e-6, max_iter=2000)
    assert all(s["converged"] for s in st)
    got, q = ctx.evaluate()
    w_all, phi_all = ctx.get_fields(), ctx.get_densities()
    orc.set_parallel(True)
    worst = 0.0
    try:
        for r, wl in enumerate(wls):
            fo = ctx.field_offset(r)
            n = wl.nsp * wl.V
            w = w_all[fo:fo + n].reshape((wl.nsp,) + wl.shape)
            phi = phi_all[fo:fo + n].reshape((wl.nsp,) + wl.shape)
            ref, qref = orc.evaluate(osys(orc, wl), w, phi[:2].sum(0).mean(), phi[2].mean())
            e = relerr(got[fo:fo + n], ref)
            worst = max(worst, e)
            assert e < TOL32 and abs(q[r] / qref - 1) < TOL32, (r, wl.L, e)
    finally:
        orc.set_parallel(False)
    say(f"  48 replicas: worst rel err {worst:.3e}")
    ctx.close()


def test_melt64_fp32_trajectory_error_on_crop(hsf, orc):
    """The FP32-propagator run of the 64^3 melt (tau 0.6, residual 1e-6): every 10th
    step the oracle evaluates phi[w^n] at the run's own fields over the full box, and the
    GPU's FP32 densities at the same fields are compared on the 32^3 crop."""
    wl = W.melt64_a8b8(tau=0.6)
    ctx = hsf.Context(wl)
    phi0 = W.initial_composition(wl)
    ctx.set_densities(phi0.ravel())
    ctx.autotune(reps=2)
    worst = 0.0
    for k in range(3):
        st, _ = ctx.step(10, tol=wl.tol, max_iter=1000)
        assert st[0]["converged"]
        w = ctx.get_fields().reshape((2,) + wl.shape)
        phi = ctx.get_densities().reshape((2,) + wl.shape)
        got, _ = ctx.evaluate()
        got = got.reshape((2,) + wl.shape)
        ref, _ = orc.evaluate(osys(orc, wl), w, phi.sum(0).mean(), 0.0)
        crop = (slice(None), slice(0, 32), slice(0, 32), slice(0, 32))
        e = max(np.max(np.abs(got[crop][i] - ref[crop][i])) / np.max(np.abs(ref[crop][i])) for i in range(2))
        worst = max(worst, e)
        say(f"[fp32 trajectory] step {10 * (k + 1)}: crop rel err {e:.3e}")
    assert worst < TOL32
    ctx.close()


def test_melt64_pair_fp32_2000_steps_error_on_crop(hsf, orc):
    """The 64^3 A8B8 pair (tau 0.6 and 1.5, one batched context, FP32 propagators,
    residual 1e-6, LB flow on) over 2000 coupled steps: every 200th step the oracle
    evaluates phi[w^n] at each replica's own fields over the full box, and the GPU's
    FP32 densities at the same fields are compared on the 32^3 crop [0, 32)^3."""
    wls = [W.melt64_a8b8(tau=0.6), W.melt64_a8b8(tau=1.5)]
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(wl).ravel() for wl in wls]))
    ctx.autotune(reps=2)
    crop = (slice(None), slice(0, 32), slice(0, 32), slice(0, 32))
    worst = 0.0
    for k in range(10):
        st, _ = ctx.step(200, tol=wls[0].tol, max_iter=1000)
        assert all(s["converged"] for s in st)
        w_all, phi_all = ctx.get_fields(), ctx.get_densities()
        got_all, _ = ctx.evaluate()
        errs = []
        for r, wl in enumerate(wls):
            o, n = ctx.field_offset(r), 2 * wl.V
            w = w_all[o:o + n].reshape((2,) + wl.shape)
            phi = phi_all[o:o + n].reshape((2,) + wl.shape)
            got = got_all[o:o + n].reshape((2,) + wl.shape)
            ref, _ = orc.evaluate(osys(orc, wl), w, phi.sum(0).mean(), 0.0)
            errs.append(max(np.max(np.abs(got[crop][i] - ref[crop][i])) / np.max(np.abs(ref[crop][i]))
                            for i in range(2)))
        worst = max(worst, max(errs))
        say(f"[fp32 pair trajectory] step {200 * (k + 1)}: crop rel err tau 0.6 {errs[0]:.3e}, tau 1.5 {errs[1]:.3e}")
    assert worst < TOL32
    ctx.close()


@pytest.mark.parametrize("hydro", [True, False], ids=["flow", "diffusive"])
def test_melt96_fp32_run_error(hsf, orc, hydro):
    """The 96^3 A4B12 melt (FP32 propagators, residual 1e-6) over 500 coupled steps,
    with the LB flow and purely diffusive (velocity zeroed): every 100th step the
    oracle evaluates phi[w^n] at the run's own fields and the GPU's FP32 densities at
    the same fields are compared over the whole box."""
    wl = W.melt96_a4b12()
    ctx = hsf.Context(wl)
    ctx.set_hydro(hydro)
    ctx.set_densities(W.initial_composition(wl).ravel())
    ctx.autotune(reps=2)
    worst = 0.0
    for k in range(5):
        st, _ = ctx.step(100, tol=wl.tol, max_iter=1000)
        assert st[0]["converged"]
        w = ctx.get_fields().reshape((2,) + wl.shape)
        phi = ctx.get_densities().reshape((2,) + wl.shape)
        got, _ = ctx.evaluate()
        got = got.reshape((2,) + wl.shape)
        ref, _ = orc.evaluate(osys(orc, wl), w, phi.sum(0).mean(), 0.0)
        e = max(np.max(np.abs(got[i] - ref[i])) / np.max(np.abs(ref[i])) for i in range(2))
        worst = max(worst, e)
        say(f"[96^3 {'flow' if hydro else 'diffusive'}] step {100 * (k + 1)}: rel err {e:.3e}")
    assert worst < TOL32
    ctx.close()


@pytest.mark.parametrize("name,steps,every", [("vesicle128_a3b9s", 100, 50), ("batch48_a3b9s", 20, 10)])
def test_solution_runs_error(hsf, orc, name, steps, every):
    """The 128^3 vesicle-forming solution and the 48 batched replicas (FP32 propagators,
    preconditioned inversion to 1e-6, LB flow on) along a run: at checkpoints the oracle
    evaluates phi[w^n] at the run's own fields (for the batch, one replica of each box
    size) and the GPU's FP32 densities at the same fields are compared."""
    wls = [W.vesicle128_a3b9s()] if name == "vesicle128_a3b9s" else W.batch48_a3b9s()
    say(f"[{name} run]")
    ctx = hsf.Context(wls)
    ctx.set_solver(precond=True)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    ctx.autotune(reps=2)
    picks = {}
    for r, w in enumerate(wls):
        picks.setdefault(w.L[0], r)
    for k in range(steps // every):
        st, _ = ctx.step(every, tol=wls[0].tol, max_iter=3000)
        assert all(s["converged"] for s in st)
        say(f" step {every * (k + 1)}:")
        check_context(hsf, orc, wls, ctx, sorted(picks.values()), TOL32)
    ctx.close()
