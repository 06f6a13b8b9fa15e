"""No kernel reads device memory before something has written it: every scenario runs
twice, once in contexts whose freshly allocated buffers hold whatever the allocator
returns and once with HSF_POISON=1 (every buffer the context allocates starts as 0xff
bytes, a NaN in FP32 and FP64), and every result must agree bit for bit.  Covers the
one-step, paired, blocked and z-streaming tilings, batched uneven replicas, the warm-start
history, the FP32 LB storage, thermal noise with the MRT collision, Crank-Nicolson steps,
observables and the FP64 refinement."""
import os
import sys

import numpy as np
import pytest

from paper_1204_2088_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def solution(L, precision, seed=3):
    return W.Workload("solution", L, W.chain(3, 9), True, W.chi_matrix(ab=25 / 12, bs=35 / 12), tau=0.8,
                      noise=0.005, seed=seed, phi_p=0.12, precision=precision)


def melt(L, precision, seed=4):
    return W.Workload("melt", L, W.chain(4, 4), False, W.chi_matrix(ab=20 / 8), tau=1.0, noise=0.01, seed=seed,
                      precision=precision)


def start(hsf, wls):
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    return ctx


def state(ctx):
    rho, u = ctx.get_flow()
    return [ctx.get_densities(), ctx.get_fields(), ctx.get_lb(), rho, u]


def scenario_paired_solution(hsf):
    wl = solution((21, 18, 16), "fp32")
    ctx = start(hsf, [wl])
    ctx.set_tile((32, 8, 4, -1))
    ctx.set_solver(precond=True)
    out = []
    ctx.invert(tol=1e-6, max_iter=2000, warm=hsf.WARM_LOCAL)
    out += [ctx.evaluate()[0]]
    ctx.set_warm(hsf.WARM_EXTRAP)
    ctx.step(3, tol=1e-6, max_iter=2000)
    out += state(ctx) + [np.array(ctx.observables()[0])]
    ctx.close()
    return out


def scenario_tilings(hsf):
    out = []
    for tile in [(32, 8, 2, 0), (16, 16, 4, 0), (8, 8, 8, 2), (64, 8, 8, 2), (16, 16, 2, -1)]:
        ctx = start(hsf, [melt((17, 12, 10), "fp64")])
        ctx.set_tile(tile)
        ctx.invert(tol=1e-8, max_iter=2000, warm=hsf.WARM_LOCAL)
        out += [ctx.evaluate()[0]]
        ctx.step(2, tol=1e-8, max_iter=2000)
        out += state(ctx)
        ctx.close()
    return out


def scenario_batch(hsf):
    wls = [solution((20, 18, 14), "fp32", seed=5), solution((12, 10, 9), "fp32", seed=6)]
    ctx = start(hsf, wls)
    ctx.set_tile((32, 8, 2, -1))
    ctx.set_warm(hsf.WARM_EXTRAP)
    ctx.step(3, tol=1e-6, max_iter=2000)
    out = state(ctx)
    ctx.close()
    return out


def scenario_noise_mrt(hsf):
    wl = melt((16, 12, 10), "fp32").with_(lb="mrt", gammas=(0.3, -0.2, 0.1))
    ctx = start(hsf, [wl])
    ctx.set_noise(cd=True, lb=True, omega=400.0, seed=9)
    ctx.step(2, tol=1e-6, max_iter=2000)
    out = state(ctx)
    ctx.close()
    return out


def scenario_cn(hsf):
    ctx = start(hsf, [melt((8, 8, 8), "fp64")])
    ctx.set_integrator(crank_nicolson=True, tol=1e-9)
    ctx.step(1, tol=1e-9, max_iter=2000)
    out = state(ctx)
    ctx.close()
    return out


def scenario_refine(hsf):
    ctx = start(hsf, [solution((14, 12, 10), "fp32")])
    ctx.set_solver(refine=True)
    ctx.invert(tol=1e-9, max_iter=2000, warm=hsf.WARM_LOCAL)
    out = [ctx.get_fields(), ctx.evaluate()[0]]
    ctx.close()
    return out


SCENARIOS = [scenario_paired_solution, scenario_tilings, scenario_batch, scenario_noise_mrt, scenario_cn,
             scenario_refine]


@pytest.mark.parametrize("scenario", SCENARIOS, ids=lambda f: f.__name__)
def test_results_do_not_depend_on_unwritten_memory(hsf, scenario):
    old = os.environ.pop("HSF_POISON", None)
    try:
        clean = scenario(hsf)
        os.environ["HSF_POISON"] = "1"
        poisoned = scenario(hsf)
    finally:
        os.environ.pop("HSF_POISON", None)
        if old is not None:
            os.environ["HSF_POISON"] = old
    assert len(clean) == len(poisoned)
    for k, (a, b) in enumerate(zip(clean, poisoned)):
        a, b = np.asarray(a), np.asarray(b)
        assert np.all(np.isfinite(a)), (scenario.__name__, k)
        assert np.array_equal(a, b), (scenario.__name__, k, float(np.nanmax(np.abs(a - b))))
    say(f"[poison] {scenario.__name__}: {len(clean)} results identical")


def test_poison_reaches_fresh_buffers(hsf):
    """The checking aid does what it says: in a fresh context with HSF_POISON=1 the
    warm-start history, which no kernel has written yet, reads back as 0xff bytes through
    the checkpoint, while the documented starting state (zero densities and fields) holds."""
    wl = melt((6, 5, 4), "fp64")
    os.environ["HSF_POISON"] = "1"
    try:
        ctx = hsf.Context([wl])
    finally:
        os.environ.pop("HSF_POISON", None)
    buf = ctx.get_state()
    nf = ctx.nsp * ctx.T
    hist = buf[buf.size - 4 * nf * 8:]   # the four history arrays close the checkpoint
    assert np.all(hist == 0xFF)
    assert np.all(ctx.get_densities() == 0.0) and np.all(ctx.get_fields() == 0.0)
    ctx.close()
