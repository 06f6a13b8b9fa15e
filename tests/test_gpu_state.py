"""Checkpoint and resume through the C ABI: a context restored from hsf_get_state's
buffer continues the run bit for bit (densities, fields and LB populations), including
the FP32 per-step scales, the extrapolating warm start's history, the thermal noise's
step word and the implicit integrator; and a buffer is refused by a context it does not
fit.
"""
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


def configure(hsf, ctx, case):
    if case == "fp32_melt_noise_extrap":
        ctx.set_warm(hsf.WARM_EXTRAP)
        ctx.set_noise(cd=True, lb=True, omega=400.0, seed=8, step=0)
    elif case == "fp64_solution_cn":
        ctx.set_integrator(True, tol=1e-11, max_newton=30, krylov_dim=40)


CASES = {
    "fp32_melt_noise_extrap": (lambda: W.Workload("ckpt", (16, 12, 10), W.chain(4, 4), False, W.chi_matrix(ab=2.5),
                                                  tau=0.8, noise=0.01, seed=1, precision="fp32", tol=1e-6), 1e-6),
    "fp64_solution_cn": (lambda: W.Workload("ckpt_sol", (10, 8, 12), W.chain(3, 9), True,
                                            W.chi_matrix(ab=25 / 12, bs=35 / 12), tau=0.8, noise=0.01, seed=2,
                                            phi_p=0.12, precision="fp64", dt=0.2), 1e-10),
}


@pytest.mark.parametrize("case", list(CASES))
def test_resume_is_bitwise(hsf, case):
    make, tol = CASES[case]
    wl = make()
    say(f"[checkpoint] {case}")
    a = hsf.Context(wl)
    configure(hsf, a, case)
    a.set_densities(W.initial_composition(wl).ravel())
    a.step(3, tol=tol, max_iter=3000)
    state = a.get_state()
    a.step(4, tol=tol, max_iter=3000)
    ref = (a.get_densities(), a.get_fields(), a.get_lb())
    a.close()

    b = hsf.Context(wl)
    configure(hsf, b, case)
    b.set_state(state)
    b.step(4, tol=tol, max_iter=3000)
    got = (b.get_densities(), b.get_fields(), b.get_lb())
    for name, x, y in zip(("densities", "fields", "populations"), got, ref):
        say(f"  {name}: max |diff| {np.max(np.abs(x - y)):.1e}")
        assert np.array_equal(x, y), name
    b.close()


def test_state_refused_by_other_contexts(hsf):
    wl = CASES["fp32_melt_noise_extrap"][0]()
    a = hsf.Context(wl)
    a.set_densities(W.initial_composition(wl).ravel())
    state = a.get_state()
    a.close()
    for other in (wl.with_(L=(16, 12, 11)), wl.with_(precision="fp64"), wl.with_(types=W.chain(3, 5))):
        c = hsf.Context(other)
        with pytest.raises(hsf.HsfError):
            c.set_state(state)
        c.close()
    c = hsf.Context(wl)
    with pytest.raises(hsf.HsfError):
        c.set_state(state[:-8])
    bad = state.copy()
    bad[:8] = 0
    with pytest.raises(hsf.HsfError):
        c.set_state(bad)
    c.close()
